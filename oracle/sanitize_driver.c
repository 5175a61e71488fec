/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE ONLY.  Calls every entry point of
 * the oracle (gfmc_oracle.h) on small lattices, including the edge cases
 * (L = 2 with coinciding start sites, odd L, M = 2, K > M, both damping
 * kernels, cap proposals, the mixed start vectors, initialisation modes),
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitizers.py) checks the oracle's memory accesses and
 * arithmetic for undefined behaviour.  Prints one line per case and a final
 * checksum; exits 0 when every result is finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "gfmc_oracle.h"

static int bad = 0;

static void check(const char* what, double v) {
  if (!isfinite(v)) {
    printf("non-finite result in %s\n", what);
    bad = 1;
  }
}

static void* xcalloc(size_t n, size_t sz) {
  void* p = calloc(n, sz);
  if (!p) {
    printf("out of memory\n");
    exit(2);
  }
  return p;
}

static double run_case(int L, int M, int K, int kernel, int proposal, int init) {
  orc_params p = {0};
  p.L = L;
  p.t = 1.0;
  p.beta = 20.0;
  p.mu = 0.0;
  p.M = M;
  p.K = K;
  p.kernel = kernel;
  p.lambda = 4.0;
  p.a = 6.0 / 0.99;
  p.b = 0.0;
  p.proposal = proposal;
  p.cone = 0.3;
  p.seed = 11;
  p.chain_id = (uint64_t)L;
  const int N = L * L * L;
  double* th = xcalloc((size_t)N, sizeof(double));
  double* ph = xcalloc((size_t)N, sizeof(double));
  orc_init_spins(&p, init, 0.25, th, ph);
  double sum = 0.0;

  double* ht = xcalloc((size_t)N * N * 2, sizeof(double));
  orc_dense_ht(&p, th, ph, ht);
  sum += ht[2];

  const int o = N / 3;
  int32_t s[7];
  orc_start_sites(L, o, s);
  double* mu = xcalloc((size_t)M * 49 * 2, sizeof(double));
  orc_moments(&p, th, ph, o, mu);
  sum += mu[(size_t)(M - 1) * 98];

  double delta[12], tn = 1.1, pn = 2.3;
  orc_deltas(&p, th, ph, o, tn, pn, delta);
  double* c4 = xcalloc((size_t)4 * M * 2, sizeof(double));
  orc_contract(M, mu, delta, c4);
  double* g = xcalloc((size_t)M, sizeof(double));
  orc_kernel_coeffs(M, kernel, p.lambda, g);
  double* G = xcalloc((size_t)4 * K * 2, sizeof(double));
  for (int q = 0; q < 4; ++q) orc_green(M, K, c4 + (size_t)q * M * 2, g, G + (size_t)q * K * 2);
  double* d = xcalloc((size_t)K * 2, sizeof(double));
  orc_det(K, p.a, G, G + (size_t)K * 2, G + (size_t)2 * K * 2, G + (size_t)3 * K * 2, d);
  double* phi = xcalloc((size_t)K, sizeof(double));
  orc_phase(K, d, phi);
  sum += orc_quadrature(K, p.beta, p.mu, p.a, p.b, phi);

  double top = 0.0;
  sum += orc_delta_seff(&p, th, ph, o, tn, pn, &top);
  sum += top;
  double* mm = xcalloc((size_t)4 * M * 2, sizeof(double));
  orc_mixed_moments(&p, th, ph, o, tn, pn, mm);
  sum += mm[1];
  sum += orc_delta_seff_mixed(&p, th, ph, o, tn, pn, NULL);

  int32_t site;
  double a1, a2, u;
  orc_propose(&p, th, ph, 5, &site, &a1, &a2, &u);
  sum += a1 + a2 + u + site;
  orc_record rec;
  orc_step(&p, th, ph, 0, -1, &rec);
  orc_step(&p, th, ph, 1, 1, &rec);
  sum += rec.dseff;
  double mag[2];
  sum += (double)orc_sweep(&p, th, ph, 0, 1, mag);
  sum += mag[0] + orc_magnetization(L, th, ph);

  uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
  orc_philox4x64_10(ctr, key, out);
  sum += orc_u01(out[0]) + (double)orc_mulhi_index(out[1], N) + orc_neighbor(L, o, 5);
  double h[2];
  orc_hopping(0.3, 0.4, 2.0, 5.0, h);
  sum += h[0] + h[1];

  printf("L=%d M=%d K=%d kernel=%d proposal=%d init=%d sum=%.17g\n", L, M, K, kernel, proposal,
         init, sum);
  check("case", sum);
  free(th); free(ph); free(ht); free(mu); free(c4); free(g); free(G); free(d); free(phi); free(mm);
  return sum;
}

int main(void) {
  double total = 0.0;
  total += run_case(2, 16, 16, 0, 0, 0);   /* doubled bonds, coinciding start sites */
  total += run_case(3, 2, 2, 1, 1, 2);     /* odd L, smallest M, Lorentz, cap, FM + random */
  total += run_case(4, 32, 64, 0, 1, 1);   /* K > M, ferromagnetic start */
  total += run_case(5, 24, 32, 1, 0, 0);   /* odd L, Lorentz, K > M */
  printf("checksum %.17g\n", total);
  return bad;
}
