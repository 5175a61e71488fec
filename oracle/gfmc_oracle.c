/*
 * gfmc_oracle.c -- plain FP64, single-threaded CPU oracle of the GFMC method
 * for the double-exchange model on the periodic simple cubic lattice.
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the HIP library is checked
 * against.  Only tests/, the smoke check and the benchmark's CPU leg load it.
 * Nothing here is shared with the HIP path.
 *
 * Each function names the passage of the paper it writes out.  Where the
 * method reaches a result with a plain definition (the Chebyshev moments
 * <j|T_n(Ht)|k>), the oracle evaluates that definition directly (one plain
 * three-term recursion per start vector, no moment doubling, no blocking);
 * where the method is an approximation (kernel-damped Green's functions,
 * the determinant, the phase and the energy integral), it follows the paper's
 * steps in the paper's order.
 *
 * Readings of passages that the paper leaves open are stated where they are
 * used (rescaling constants, kernel, node set, phase branch, RNG).
 */
#include "gfmc_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).        */
/* The paper only says "rand()"; a counter-based generator makes every draw  */
/* addressable by (key, counter), so CPU and GPU draw identical streams.     */
/* ------------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  /* Round multipliers and Weyl key increments of Philox-4x64 as published. */
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mul128(M0, x0, &hi0, &lo0);
    mul128(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

int64_t orc_mulhi_index(uint64_t r, int64_t n) {
  unsigned __int128 p = (unsigned __int128)r * (unsigned __int128)(uint64_t)n;
  return (int64_t)(uint64_t)(p >> 64);
}

double orc_u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* Counter purposes: 1 = proposal, 2 = per-site initial spin, 3 = selection
 * of randomised sites for the "ferromagnet plus a random fraction" start. */
static void draw(const orc_params* p, uint64_t c0, uint64_t purpose, uint64_t out[4]) {
  uint64_t ctr[4] = {c0, purpose, 0, 0};
  uint64_t key[2] = {p->seed, p->chain_id};
  orc_philox4x64_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Model: Section 2.1, infinite-Hund double-exchange Hamiltonian.            */
/* ------------------------------------------------------------------------ */
int32_t orc_neighbor(int32_t L, int32_t i, int32_t d) {
  int32_t x = i % L, y = (i / L) % L, z = i / (L * L);
  switch (d) {
    case 0: x = (x + 1) % L; break;
    case 1: x = (x + L - 1) % L; break;
    case 2: y = (y + 1) % L; break;
    case 3: y = (y + L - 1) % L; break;
    case 4: z = (z + 1) % L; break;
    default: z = (z + L - 1) % L; break;
  }
  return x + L * (y + L * z);
}

/* Hopping amplitude of the J_H -> infinity limit (equation "ht"):
 *   t_ij = cos((th_i - th_j)/2) cos((ph_i - ph_j)/2)
 *        + i cos((th_i + th_j)/2) sin((ph_i - ph_j)/2).                     */
void orc_hopping(double th_i, double ph_i, double th_j, double ph_j, double out[2]) {
  out[0] = cos(0.5 * (th_i - th_j)) * cos(0.5 * (ph_i - ph_j));
  out[1] = cos(0.5 * (th_i + th_j)) * sin(0.5 * (ph_i - ph_j));
}

static cplx hop(double th_i, double ph_i, double th_j, double ph_j) {
  double h[2];
  orc_hopping(th_i, ph_i, th_j, ph_j, h);
  return h[0] + I * h[1];
}

/* Matrix element <i|H|j> = -t t_ij for every nearest-neighbour bond; the
 * model is spinless after the infinite-Hund projection, one orbital per
 * site, so H is N x N.  Bonds are added per direction, so for L = 2 the two
 * bonds joining the same pair of sites both count.  Rescaled Ht = (H - b)/a
 * (Section 2.2, around the Chebyshev expansion). */
void orc_dense_ht(const orc_params* p, const double* th, const double* ph, double* ht) {
  const int32_t L = p->L, N = L * L * L;
  memset(ht, 0, sizeof(double) * 2 * (size_t)N * (size_t)N);
  for (int32_t i = 0; i < N; ++i) {
    ht[2 * ((size_t)i * N + i)] += -p->b / p->a;
    for (int32_t d = 0; d < 6; ++d) {
      int32_t j = orc_neighbor(L, i, d);
      cplx v = -(p->t / p->a) * hop(th[i], ph[i], th[j], ph[j]);
      ht[2 * ((size_t)i * N + j)] += creal(v);
      ht[2 * ((size_t)i * N + j) + 1] += cimag(v);
    }
  }
}

/* Ht in a 6-entry-per-row neighbour list (the matrix is never stored by the
 * HIP path; here it is the plainest way to apply Ht). */
static void build_rows(const orc_params* p, const double* th, const double* ph, int32_t* col,
                       cplx* val) {
  const int32_t L = p->L, N = L * L * L;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t d = 0; d < 6; ++d) {
      int32_t j = orc_neighbor(L, i, d);
      col[6 * i + d] = j;
      val[6 * i + d] = -(p->t / p->a) * hop(th[i], ph[i], th[j], ph[j]);
    }
}

static void apply_ht(int32_t N, double diag, const int32_t* col, const cplx* val, const cplx* x,
                     cplx* y) {
  for (int32_t i = 0; i < N; ++i) {
    cplx s = diag * x[i];
    for (int32_t d = 0; d < 6; ++d) s += val[6 * i + d] * x[col[6 * i + d]];
    y[i] = s;
  }
}

void orc_start_sites(int32_t L, int32_t o, int32_t s[7]) {
  s[0] = o;
  for (int32_t d = 0; d < 6; ++d) s[1 + d] = orc_neighbor(L, o, d);
}

/* Local moments mu_n^{jk} = <s_j|T_n(Ht)|s_k> (Section 2.2, definition of the
 * moments), evaluated from the definition: |a_0> = |s_k>, |a_1> = Ht|a_0>,
 * |a_n> = 2 Ht|a_{n-1}> - |a_{n-2}> (equation "recursive"), and
 * mu_n^{jk} = <s_j|a_n> = a_n[s_j].  No moment doubling: the HIP path's
 * doubling identity is checked against this. */
void orc_moments(const orc_params* p, const double* th, const double* ph, int32_t o, double* mu) {
  const int32_t L = p->L, N = L * L * L, M = p->M;
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * 6 * (size_t)N);
  cplx* val = (cplx*)malloc(sizeof(cplx) * 6 * (size_t)N);
  cplx* a0 = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  cplx* a1 = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  cplx* a2 = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  build_rows(p, th, ph, col, val);
  const double diag = -p->b / p->a;
  int32_t s[7];
  orc_start_sites(L, o, s);
  for (int32_t k = 0; k < 7; ++k) {
    for (int32_t i = 0; i < N; ++i) a0[i] = 0.0;
    a0[s[k]] = 1.0;
    for (int32_t j = 0; j < 7; ++j) {
      mu[2 * ((0 * 7 + j) * 7 + k)] = creal(a0[s[j]]);
      mu[2 * ((0 * 7 + j) * 7 + k) + 1] = cimag(a0[s[j]]);
    }
    if (M < 2) continue;
    apply_ht(N, diag, col, val, a0, a1);
    for (int32_t j = 0; j < 7; ++j) {
      mu[2 * ((1 * 7 + j) * 7 + k)] = creal(a1[s[j]]);
      mu[2 * ((1 * 7 + j) * 7 + k) + 1] = cimag(a1[s[j]]);
    }
    cplx *prev = a0, *cur = a1, *next = a2;
    for (int32_t n = 2; n < M; ++n) {
      apply_ht(N, diag, col, val, cur, next);
      for (int32_t i = 0; i < N; ++i) next[i] = 2.0 * next[i] - prev[i];
      for (int32_t j = 0; j < 7; ++j) {
        mu[2 * (((size_t)n * 7 + j) * 7 + k)] = creal(next[s[j]]);
        mu[2 * (((size_t)n * 7 + j) * 7 + k) + 1] = cimag(next[s[j]]);
      }
      cplx* tmp = prev; prev = cur; cur = next; next = tmp;
    }
  }
  free(col); free(val); free(a0); free(a1); free(a2);
}

/* ------------------------------------------------------------------------ */
/* Section 2.2: the local change Delta = H' - H and the 2x2 reduction.       */
/* Delta is nonzero only in row and column o; |v> = Delta|o> collects the    */
/* six bond changes.  The algorithm box writes "H - H'", the derivation and   */
/* the update "H <- H + Delta" need H' - H, which is used here.              */
/* ------------------------------------------------------------------------ */
void orc_deltas(const orc_params* p, const double* th, const double* ph, int32_t o,
                double th_new, double ph_new, double* delta) {
  for (int32_t d = 0; d < 6; ++d) {
    int32_t n = orc_neighbor(p->L, o, d);
    cplx h_new = -p->t * hop(th[n], ph[n], th_new, ph_new);
    cplx h_old = -p->t * hop(th[n], ph[n], th[o], ph[o]);
    cplx dd = h_new - h_old;
    delta[2 * d] = creal(dd);
    delta[2 * d + 1] = cimag(dd);
  }
}

/* Moments of the four Green's functions needed by equation "d_z_green":
 *   mu^{oo} = mu^{o o},  mu^{ov} = sum_k delta_k mu^{o k},
 *   mu^{vo} = sum_j conj(delta_j) mu^{j o},
 *   mu^{vv} = sum_{jk} conj(delta_j) delta_k mu^{j k},
 * with |v> = sum_k delta_k |n_k>. */
void orc_contract(int32_t M, const double* mu, const double* delta, double* out) {
  for (int32_t n = 0; n < M; ++n) {
    cplx m[7][7];
    for (int32_t j = 0; j < 7; ++j)
      for (int32_t k = 0; k < 7; ++k)
        m[j][k] = mu[2 * (((size_t)n * 7 + j) * 7 + k)] +
                  I * mu[2 * (((size_t)n * 7 + j) * 7 + k) + 1];
    cplx dl[6];
    for (int32_t d = 0; d < 6; ++d) dl[d] = delta[2 * d] + I * delta[2 * d + 1];
    cplx oo = m[0][0], ov = 0, vo = 0, vv = 0;
    for (int32_t k = 0; k < 6; ++k) ov += dl[k] * m[0][1 + k];
    for (int32_t j = 0; j < 6; ++j) vo += conj(dl[j]) * m[1 + j][0];
    for (int32_t j = 0; j < 6; ++j)
      for (int32_t k = 0; k < 6; ++k) vv += conj(dl[j]) * dl[k] * m[1 + j][1 + k];
    cplx r[4] = {oo, ov, vo, vv};
    for (int32_t s = 0; s < 4; ++s) {
      out[2 * ((size_t)s * M + n)] = creal(r[s]);
      out[2 * ((size_t)s * M + n) + 1] = cimag(r[s]);
    }
  }
}

/* Damping kernels (Section 2.2).  The paper names the Lorentz kernel
 * g_n = sinh(lambda (1 - n/M)) / sinh(lambda) without a lambda; the Jackson
 * kernel of the kernel-polynomial review it cites is the default here:
 * g_n = [(M - n + 1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1). */
void orc_kernel_coeffs(int32_t M, int32_t kind, double lambda, double* g) {
  for (int32_t n = 0; n < M; ++n) {
    if (kind == 1) {
      g[n] = sinh(lambda * (1.0 - (double)n / M)) / sinh(lambda);
    } else {
      double q = PI / (M + 1.0);
      g[n] = ((M - n + 1.0) * cos(q * n) + sin(q * n) * cos(q) / sin(q)) / (M + 1.0);
    }
  }
}

/* Equations "green" and "green_short": at w_k = cos(th_k), th_k = pi(k+1/2)/K,
 *   Gt(w_k + i0) = (2i / sin th_k) sum_{n<M} mu'_n exp(-i n th_k),
 * mu'_0 = g_0 mu_0 / 2, mu'_n = g_n mu_n.  Evaluated by direct O(MK)
 * summation (the method evaluates the same sum by FFT).  Complex moments
 * (off-diagonal elements) enter linearly. */
void orc_green(int32_t M, int32_t K, const double* mu, const double* g, double* G) {
  for (int32_t k = 0; k < K; ++k) {
    double thk = PI * (k + 0.5) / K;
    cplx s = 0;
    for (int32_t n = 0; n < M; ++n) {
      cplx m = g[n] * (mu[2 * n] + I * mu[2 * n + 1]);
      if (n == 0) m *= 0.5;
      s += m * (cos(n * thk) - I * sin(n * thk));
    }
    cplx Gk = 2.0 * I * s / sin(thk);
    G[2 * k] = creal(Gk);
    G[2 * k + 1] = cimag(Gk);
  }
}

/* Equation "d_z_green" with physical G = Gt / a (G is the resolvent of H, the
 * moments are those of Ht = (H - b)/a). */
void orc_det(int32_t K, double a, const double* Goo, const double* Gov, const double* Gvo,
             const double* Gvv, double* d) {
  for (int32_t k = 0; k < K; ++k) {
    cplx goo = (Goo[2 * k] + I * Goo[2 * k + 1]) / a;
    cplx gov = (Gov[2 * k] + I * Gov[2 * k + 1]) / a;
    cplx gvo = (Gvo[2 * k] + I * Gvo[2 * k + 1]) / a;
    cplx gvv = (Gvv[2 * k] + I * Gvv[2 * k + 1]) / a;
    cplx dk = (1.0 + gov) * (1.0 + gvo) - goo * gvv;
    d[2 * k] = creal(dk);
    d[2 * k + 1] = cimag(dk);
  }
}

/* Im log d(E + i0) on the nodes, on the branch that is 0 below the spectrum
 * (the integration by parts leading to equation "d_seff2" needs it): start
 * from the lowest node (k = K-1) and add the principal argument of each
 * ratio d_k / d_{k+1}. */
void orc_phase(int32_t K, const double* d, double* phi) {
  phi[K - 1] = atan2(d[2 * (K - 1) + 1], d[2 * (K - 1)]);
  for (int32_t k = K - 2; k >= 0; --k) {
    cplx r = (d[2 * k] + I * d[2 * k + 1]) * conj(d[2 * (k + 1)] + I * d[2 * (k + 1) + 1]);
    phi[k] = phi[k + 1] + carg(r);
  }
}

static double fermi(double beta, double e, double mu) {
  double x = beta * (e - mu);
  if (x > 0) {
    double q = exp(-x);
    return q / (1.0 + q);
  }
  return 1.0 / (1.0 + exp(x));
}

/* Equation "d_seff2": Delta S = (beta/pi) int f(E) Im log d(E+i0) dE with
 * E = a w + b and Gauss-Chebyshev quadrature on the same K nodes:
 * int F(w) dw ~ (pi/K) sum_k F(w_k) sin th_k. */
double orc_quadrature(int32_t K, double beta, double mu, double a, double b, const double* phi) {
  double s = 0;
  for (int32_t k = 0; k < K; ++k) {
    double thk = PI * (k + 0.5) / K;
    double e = a * cos(thk) + b;
    s += fermi(beta, e, mu) * sin(thk) * phi[k];
  }
  return beta * a / K * s;
}

/* Algorithm 1, body of the inner loop (from the change of the spin to
 * Delta S_eff): deltas, local moments, kernel, four Green's functions,
 * determinant, phase, energy integral. */
double orc_delta_seff(const orc_params* p, const double* th, const double* ph, int32_t o,
                      double th_new, double ph_new, double* phase_top) {
  const int32_t M = p->M, K = p->K;
  double delta[12];
  orc_deltas(p, th, ph, o, th_new, ph_new, delta);
  double* mu = (double*)malloc(sizeof(double) * 2 * 49 * (size_t)M);
  double* m4 = (double*)malloc(sizeof(double) * 2 * 4 * (size_t)M);
  double* g = (double*)malloc(sizeof(double) * (size_t)M);
  double* G = (double*)malloc(sizeof(double) * 2 * 4 * (size_t)K);
  double* d = (double*)malloc(sizeof(double) * 2 * (size_t)K);
  double* phi = (double*)malloc(sizeof(double) * (size_t)K);
  orc_moments(p, th, ph, o, mu);
  orc_contract(M, mu, delta, m4);
  orc_kernel_coeffs(M, p->kernel, p->lambda, g);
  for (int32_t s = 0; s < 4; ++s) orc_green(M, K, m4 + 2 * (size_t)s * M, g, G + 2 * (size_t)s * K);
  orc_det(K, p->a, G, G + 2 * (size_t)K, G + 4 * (size_t)K, G + 6 * (size_t)K, d);
  orc_phase(K, d, phi);
  double ds = orc_quadrature(K, p->beta, p->mu, p->a, p->b, phi);
  if (phase_top) *phase_top = phi[0];
  free(mu); free(m4); free(g); free(G); free(d); free(phi);
  return ds;
}

/* ------------------------------------------------------------------------ */
/* Section 2.2, off-diagonal elements from mixed diagonal elements: the four  */
/* start vectors |o>, |v>, |o> + |v>, |o> + i|v> (|v> = sum_d delta_d |n_d>), */
/* their diagonal moments, and G_ov, G_vo from the diagonal Green's          */
/* functions of the mixed vectors.                                            */
/* ------------------------------------------------------------------------ */

/* mu[(s * M + n) * 2 + {0,1}] = <a_s|T_n(Ht)|a_s> for the start vectors
 * a_0 = |o>, a_1 = |v>, a_2 = |o> + |v>, a_3 = |o> + i|v>, from the
 * definition: plain three-term recursion (equation "recursive") on the full
 * vector, no doubling.  The imaginary parts vanish up to rounding (Ht is
 * Hermitian) and are returned for checking. */
void orc_mixed_moments(const orc_params* p, const double* th, const double* ph, int32_t o,
                       double th_new, double ph_new, double* mu) {
  const int32_t L = p->L, N = L * L * L, M = p->M;
  double delta[12];
  orc_deltas(p, th, ph, o, th_new, ph_new, delta);
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * 6 * (size_t)N);
  cplx* val = (cplx*)malloc(sizeof(cplx) * 6 * (size_t)N);
  cplx* st = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  cplx* a0 = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  cplx* a1 = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  cplx* a2 = (cplx*)malloc(sizeof(cplx) * (size_t)N);
  build_rows(p, th, ph, col, val);
  const double diag = -p->b / p->a;
  const cplx co[4] = {1.0, 0.0, 1.0, 1.0};     /* weight of |o> */
  const cplx cv[4] = {0.0, 1.0, 1.0, I};       /* weight of |v> */
  for (int32_t s = 0; s < 4; ++s) {
    for (int32_t i = 0; i < N; ++i) st[i] = 0.0;
    st[o] += co[s];
    for (int32_t d = 0; d < 6; ++d)
      st[orc_neighbor(L, o, d)] += cv[s] * (delta[2 * d] + I * delta[2 * d + 1]);
    cplx *prev = a0, *cur = a1, *next = a2;
    for (int32_t i = 0; i < N; ++i) prev[i] = st[i];
    for (int32_t n = 0; n < M; ++n) {
      cplx* an;
      if (n == 0) {
        an = prev;
      } else if (n == 1) {
        apply_ht(N, diag, col, val, prev, cur);
        an = cur;
      } else {
        apply_ht(N, diag, col, val, cur, next);
        for (int32_t i = 0; i < N; ++i) next[i] = 2.0 * next[i] - prev[i];
        cplx* tmp = prev; prev = cur; cur = next; next = tmp;
        an = cur;
      }
      cplx m = 0;
      for (int32_t i = 0; i < N; ++i) m += conj(st[i]) * an[i];
      mu[2 * ((size_t)s * M + n)] = creal(m);
      mu[2 * ((size_t)s * M + n) + 1] = cimag(m);
    }
  }
  free(col); free(val); free(st); free(a0); free(a1); free(a2);
}

/* Delta S_eff through the mixed start vectors: Gt_aa for a = o, v, o+v, o+iv
 * from their diagonal moments (equation "green_short", direct sum), then
 *   G_ov = [G_{o+v} - G_oo - G_vv + i (G_oo + G_vv - G_{o+iv})] / 2,
 *   G_vo = [G_{o+v} - G_oo - G_vv + i (G_{o+iv} - G_oo - G_vv)] / 2,
 * and the determinant, phase and energy integral as for the site vectors. */
double orc_delta_seff_mixed(const orc_params* p, const double* th, const double* ph, int32_t o,
                            double th_new, double ph_new, double* phase_top) {
  const int32_t M = p->M, K = p->K;
  double* mu = (double*)malloc(sizeof(double) * 2 * 4 * (size_t)M);
  double* g = (double*)malloc(sizeof(double) * (size_t)M);
  double* G = (double*)malloc(sizeof(double) * 2 * 4 * (size_t)K);
  double* Gx = (double*)malloc(sizeof(double) * 2 * 2 * (size_t)K);
  double* d = (double*)malloc(sizeof(double) * 2 * (size_t)K);
  double* phi = (double*)malloc(sizeof(double) * (size_t)K);
  orc_mixed_moments(p, th, ph, o, th_new, ph_new, mu);
  for (int32_t i = 0; i < 4 * M; ++i) mu[2 * i + 1] = 0.0;   /* diagonal: real */
  orc_kernel_coeffs(M, p->kernel, p->lambda, g);
  for (int32_t s = 0; s < 4; ++s) orc_green(M, K, mu + 2 * (size_t)s * M, g, G + 2 * (size_t)s * K);
  for (int32_t k = 0; k < K; ++k) {
    cplx goo = G[2 * k] + I * G[2 * k + 1];
    cplx gvv = G[2 * ((size_t)K + k)] + I * G[2 * ((size_t)K + k) + 1];
    cplx gp = G[2 * (2 * (size_t)K + k)] + I * G[2 * (2 * (size_t)K + k) + 1];
    cplx gi = G[2 * (3 * (size_t)K + k)] + I * G[2 * (3 * (size_t)K + k) + 1];
    cplx gov = 0.5 * (gp - goo - gvv + I * (goo + gvv - gi));
    cplx gvo = 0.5 * (gp - goo - gvv + I * (gi - goo - gvv));
    Gx[2 * k] = creal(gov);
    Gx[2 * k + 1] = cimag(gov);
    Gx[2 * ((size_t)K + k)] = creal(gvo);
    Gx[2 * ((size_t)K + k) + 1] = cimag(gvo);
  }
  orc_det(K, p->a, G, Gx, Gx + 2 * (size_t)K, G + 2 * (size_t)K, d);
  orc_phase(K, d, phi);
  double ds = orc_quadrature(K, p->beta, p->mu, p->a, p->b, phi);
  if (phase_top) *phase_top = phi[0];
  free(mu); free(g); free(G); free(Gx); free(d); free(phi);
  return ds;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: proposals, Metropolis, sweeps, magnetization.                 */
/* ------------------------------------------------------------------------ */
static void sphere_angles(double ua, double ub, double* th, double* ph) {
  *th = acos(1.0 - 2.0 * ua);
  *ph = 2.0 * PI * ub;
}

/* "Randomly choose site o and change the spin randomly": site uniform, new
 * direction uniform on the sphere, or uniform on the cap of half-angle
 * `cone` around the old direction (both proposals are symmetric). */
void orc_propose(const orc_params* p, const double* th, const double* ph, int64_t index,
                 int32_t* site, double* th_new, double* ph_new, double* u) {
  const int64_t N = (int64_t)p->L * p->L * p->L;
  uint64_t r[4];
  draw(p, (uint64_t)index, 1, r);
  int32_t o = (int32_t)orc_mulhi_index(r[0], N);
  double ua = orc_u01(r[1]), ub = orc_u01(r[2]);
  *u = orc_u01(r[3]);
  *site = o;
  if (p->proposal == 1) {
    double t0 = th[o], p0 = ph[o];
    double S[3] = {sin(t0) * cos(p0), sin(t0) * sin(p0), cos(t0)};
    double e1[3] = {cos(t0) * cos(p0), cos(t0) * sin(p0), -sin(t0)};
    double e2[3] = {-sin(p0), cos(p0), 0.0};
    double ca = 1.0 - (1.0 - cos(p->cone)) * ua;
    double sa = sqrt(fmax(0.0, (1.0 - ca) * (1.0 + ca)));
    double psi = 2.0 * PI * ub;
    double Sn[3];
    for (int q = 0; q < 3; ++q) Sn[q] = ca * S[q] + sa * (cos(psi) * e1[q] + sin(psi) * e2[q]);
    *th_new = atan2(sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1]), Sn[2]);
    double pn = atan2(Sn[1], Sn[0]);
    if (pn < 0) pn += 2.0 * PI;
    *ph_new = pn;
  } else {
    sphere_angles(ua, ub, th_new, ph_new);
  }
}

void orc_step(const orc_params* p, double* th, double* ph, int64_t index, int32_t force,
              orc_record* rec) {
  int32_t o;
  double tn, pn, u, top = 0;
  orc_propose(p, th, ph, index, &o, &tn, &pn, &u);
  double ds = orc_delta_seff(p, th, ph, o, tn, pn, &top);
  /* Metropolis: accept when exp(-Delta S) > u, i.e. Delta S <= 0 or u < exp(-Delta S). */
  int32_t own = (ds <= 0.0 || u < exp(-ds)) ? 1 : 0;
  int32_t acc = force < 0 ? own : (force ? 1 : 0);
  if (rec) {
    rec->index = index; rec->site = o; rec->own = own; rec->accepted = acc;
    rec->theta_old = th[o]; rec->phi_old = ph[o]; rec->theta_new = tn; rec->phi_new = pn;
    rec->dseff = ds; rec->u = u; rec->phase_top = top;
  }
  if (acc) { th[o] = tn; ph[o] = pn; }
}

double orc_magnetization(int32_t L, const double* th, const double* ph) {
  const int32_t N = L * L * L;
  double sx = 0, sy = 0, sz = 0;
  for (int32_t i = 0; i < N; ++i) {
    sx += sin(th[i]) * cos(ph[i]);
    sy += sin(th[i]) * sin(ph[i]);
    sz += cos(th[i]);
  }
  return sqrt(sx * sx + sy * sy + sz * sz) / N;
}

/* Sweep s consists of the N proposals with counter values s*N + j. */
int64_t orc_sweep(const orc_params* p, double* th, double* ph, int64_t sweep0, int32_t nsweeps,
                  double* magnetization) {
  const int64_t N = (int64_t)p->L * p->L * p->L;
  int64_t accepted = 0;
  for (int32_t s = 0; s < nsweeps; ++s) {
    for (int64_t j = 0; j < N; ++j) {
      orc_record rec;
      orc_step(p, th, ph, (sweep0 + s) * N + j, -1, &rec);
      accepted += rec.accepted;
    }
    if (magnetization) magnetization[s] = orc_magnetization(p->L, th, ph);
  }
  return accepted;
}

void orc_init_spins(const orc_params* p, int32_t mode, double frac, double* th, double* ph) {
  const int64_t N = (int64_t)p->L * p->L * p->L;
  if (mode == 0) {
    for (int64_t i = 0; i < N; ++i) {
      uint64_t r[4];
      draw(p, (uint64_t)i, 2, r);
      sphere_angles(orc_u01(r[0]), orc_u01(r[1]), &th[i], &ph[i]);
    }
    return;
  }
  for (int64_t i = 0; i < N; ++i) { th[i] = 0.0; ph[i] = 0.0; }
  if (mode != 2) return;
  /* exactly floor(frac*N) distinct sites, chosen by a partial Fisher-Yates
   * shuffle, each redrawn uniformly on the sphere */
  int64_t nr = (int64_t)floor(frac * (double)N);
  if (nr > N) nr = N;
  if (nr < 0) nr = 0;
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  for (int64_t i = 0; i < N; ++i) perm[i] = i;
  for (int64_t k = 0; k < nr; ++k) {
    uint64_t r[4];
    draw(p, (uint64_t)k, 3, r);
    int64_t j = k + orc_mulhi_index(r[0], N - k);
    int64_t tmp = perm[k]; perm[k] = perm[j]; perm[j] = tmp;
  }
  for (int64_t k = 0; k < nr; ++k) {
    int64_t i = perm[k];
    uint64_t r[4];
    draw(p, (uint64_t)i, 2, r);
    sphere_angles(orc_u01(r[0]), orc_u01(r[1]), &th[i], &ph[i]);
  }
  free(perm);
}
