/*
 * gfmc_oracle.h -- plain FP64 CPU oracle for the O(N) Green-function-based
 * Monte Carlo (GFMC) method applied to the 3D double-exchange model
 * (Zhang, Yamagiwa, Yunoki, "A Study of Parallelizing O(N) Green-Function-Based
 * Monte Carlo Method for Many Fermions Coupled with Classical Degrees of Freedom").
 *
 * TEST INFRASTRUCTURE ONLY.  This header and its implementation are the
 * correctness reference for the HIP library in paper_1303_6016_amd/.  Only the
 * tests, the smoke check and the CPU leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the HIP path.
 *
 * Single-threaded, no blocking, no fusion: every function follows one passage
 * of the paper (cited per function in gfmc_oracle.c).
 *
 * Conventions (shared *by definition* with the HIP path, implemented twice):
 *   sites        i = x + L*(y + L*z), periodic, L >= 2
 *   directions   d = 0..5 : +x, -x, +y, -y, +z, -z
 *   start labels j = 0..6 : o, n_{+x}, n_{-x}, n_{+y}, n_{-y}, n_{+z}, n_{-z}
 *   moments      mu[n][j][k][2] = <j| T_n(Ht) |k>   (re, im), n = 0..M-1
 *   Hamiltonian  H_{i,nb} = -t * t_{i,nb}, Ht = (H - b) / a
 */
#ifndef GFMC_ORACLE_H
#define GFMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t L;          /* linear size, N = L^3                               */
  double t;           /* hopping scale                                      */
  double beta, mu;    /* inverse temperature, chemical potential            */
  int32_t M;          /* number of Chebyshev moments (even, >= 2)           */
  int32_t K;          /* number of energy nodes (>= M)                      */
  int32_t kernel;     /* 0 = Jackson, 1 = Lorentz                           */
  double lambda;      /* Lorentz parameter                                  */
  double a, b;        /* spectral rescaling Ht = (H - b)/a                  */
  int32_t proposal;   /* 0 = uniform on the sphere, 1 = uniform on a cap    */
  double cone;        /* cap half-angle (rad)                               */
  uint64_t seed, chain_id;   /* Philox key                                  */
} orc_params;

typedef struct {
  int64_t index;      /* proposal counter value (sweep*N + j)              */
  int32_t site;       /* proposed site o                                   */
  int32_t own;        /* Metropolis decision taken from (dseff, u)         */
  int32_t accepted;   /* decision applied (own unless forced)              */
  double theta_old, phi_old, theta_new, phi_new;
  double dseff, u;
  double phase_top;   /* continuous phase at the highest node (diagnostic) */
} orc_record;

/* Philox4x64-10 block function (Salmon et al., SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* floor(r * n / 2^64): uniform integer in [0, n) from a 64-bit draw. */
int64_t orc_mulhi_index(uint64_t r, int64_t n);
/* (r >> 11) * 2^-53: uniform double in [0, 1). */
double orc_u01(uint64_t r);

/* Lattice neighbour of site i in direction d. */
int32_t orc_neighbor(int32_t L, int32_t i, int32_t d);
/* Hopping amplitude t_ij of the infinite-Hund limit, written out from its angles. */
void orc_hopping(double th_i, double ph_i, double th_j, double ph_j, double out[2]);
/* Dense rescaled Hamiltonian Ht (N x N complex, row-major, [2] = re/im). */
void orc_dense_ht(const orc_params* p, const double* th, const double* ph, double* ht);

/* Start-vector sites: s[0] = o, s[1+d] = neighbour of o in direction d. */
void orc_start_sites(int32_t L, int32_t o, int32_t s[7]);
/* Local Chebyshev moments mu[n][j][k] = <s_j|T_n(Ht)|s_k>, n < M. */
void orc_moments(const orc_params* p, const double* th, const double* ph, int32_t o,
                 double* mu /* [M][7][7][2] */);

/* Hopping changes delta_d = Delta_{n_d,o} = H'_{n_d,o} - H_{n_d,o}. */
void orc_deltas(const orc_params* p, const double* th, const double* ph, int32_t o,
                double th_new, double ph_new, double* delta /* [6][2] */);
/* Moments of the 2x2 block: out[s][n][2], s = 0:oo, 1:ov, 2:vo, 3:vv. */
void orc_contract(int32_t M, const double* mu, const double* delta, double* out);
/* Kernel coefficients g_n, n < M. */
void orc_kernel_coeffs(int32_t M, int32_t kind, double lambda, double* g);
/* Rescaled Green's function Gt(w_k + i0) at the K Chebyshev nodes from moments
 * mu_n (complex), by direct summation. */
void orc_green(int32_t M, int32_t K, const double* mu /* [M][2] */, const double* g,
               double* G /* [K][2] */);
/* d_k = (1 + G_ov)(1 + G_vo) - G_oo G_vv for physical G = Gt / a. */
void orc_det(int32_t K, double a, const double* Goo, const double* Gov, const double* Gvo,
             const double* Gvv, double* d /* [K][2] */);
/* Continuous phase of d along the nodes, anchored at the lowest node. */
void orc_phase(int32_t K, const double* d, double* phi);
/* Fermi-weighted energy integral of the phase (Gauss-Chebyshev on the nodes). */
double orc_quadrature(int32_t K, double beta, double mu, double a, double b, const double* phi);
/* Full Delta S_eff for moving spin o to (th_new, ph_new); phase_top optional. */
double orc_delta_seff(const orc_params* p, const double* th, const double* ph, int32_t o,
                      double th_new, double ph_new, double* phase_top);

/* The paper's mixed start vectors |o>, |v>, |o>+|v>, |o>+i|v> (Section 2.2,
 * off-diagonal Green's functions from mixed diagonal elements): diagonal
 * moments mu[4][M][2] by plain recursion on full vectors, and Delta S_eff
 * with G_ov, G_vo formed from the four diagonal Green's functions. */
void orc_mixed_moments(const orc_params* p, const double* th, const double* ph, int32_t o,
                       double th_new, double ph_new, double* mu);
double orc_delta_seff_mixed(const orc_params* p, const double* th, const double* ph, int32_t o,
                            double th_new, double ph_new, double* phase_top);

/* Proposal draw for counter value `index`: site, new angles, acceptance draw. */
void orc_propose(const orc_params* p, const double* th, const double* ph, int64_t index,
                 int32_t* site, double* th_new, double* ph_new, double* u);
/* One Metropolis step; force: -1 own decision, 0 reject, 1 accept. */
void orc_step(const orc_params* p, double* th, double* ph, int64_t index, int32_t force,
              orc_record* rec);
/* nsweeps sweeps of N proposals starting at sweep `sweep0`; |m| per sweep. */
int64_t orc_sweep(const orc_params* p, double* th, double* ph, int64_t sweep0, int32_t nsweeps,
                  double* magnetization);
/* |sum_i S_i| / N */
double orc_magnetization(int32_t L, const double* th, const double* ph);

/* Spin initialisation: 0 uniform sphere, 1 ferromagnetic, 2 FM + floor(frac*N) random. */
void orc_init_spins(const orc_params* p, int32_t mode, double frac, double* th, double* ph);

#ifdef __cplusplus
}
#endif
#endif
