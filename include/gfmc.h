/*
 * gfmc.h -- C ABI of the MI355X (gfx950) library for the O(N) Green-function-
 * based Monte Carlo (GFMC) method on the 3D double-exchange model (Zhang,
 * Yamagiwa, Yunoki, arXiv:1303.6016).
 *
 * What the library computes (Section 2 of the paper):
 *   model   H = -t sum_<ij> t_ij c_i^+ c_j + h.c. in the infinite-Hund limit,
 *           t_ij from the polar/azimuthal angles of the classical spins
 *           (equation "ht"), periodic L x L x L simple cubic lattice;
 *   moments mu_n^{jk} = <j|T_n(Ht)|k> of Ht = (H - b)/a for the 7 sites touched
 *           by a local spin change (site o and its 6 neighbours), from M/2 steps
 *           of the three-term recursion (equation "recursive") with moment
 *           doubling (equation "mu2");
 *   Delta S_eff from the kernel-damped local Green's functions (equations
 *           "green", "green_short"/"green_fft"), the 2x2 determinant
 *           (equation "d_z_green") and the Fermi-weighted phase integral
 *           (equation "d_seff2");
 *   Metropolis sweeps of Algorithm 1 with the magnetization |sum_i S_i|/N.
 *
 * Conventions:
 *   site index      i = x + L*(y + L*z)
 *   directions      d = 0..5 : +x, -x, +y, -y, +z, -z
 *   start labels    j = 0..6 : o, then the neighbour of o in direction j-1
 *   moment layout   mu[n][j][k][2] (re, im), n = 0..M-1, row-major, FP64
 *   random numbers  Philox4x64-10, key (seed, chain_id); counter
 *                   (sweep*N + j, 1, 0, 0) for proposal j of a sweep,
 *                   (i, 2, 0, 0) for the initial spin of site i,
 *                   (k, 3, 0, 0) for the k-th pick of randomised sites.
 *
 * Ownership: the caller allocates and owns all host arrays, all device memory
 * (the workspace passed to gfmc_chain_create / gfmc_batch_create) and the HIP
 * stream.  The library copies host inputs, writes only into caller buffers,
 * and owns only the opaque handles.  Destroying a handle never frees caller
 * memory.
 *
 * Errors: every entry point returns gfmc_status and never throws or aborts.
 * Invalid input returns GFMC_EINVAL with the state unchanged; the reason is
 * available from gfmc_last_error() (thread-local).  HIP failures return
 * GFMC_EDEVICE.
 *
 * Asynchrony: device work is enqueued on the handle's stream.  Calls that
 * return host data (moments, delta_seff, step records, spins, sweep results)
 * synchronize that stream before returning.
 *
 * Threading: a chain or batch handle is used by one caller thread at a time.
 *
 * Restrictions of the device path (EINVAL otherwise):
 *   L even, 2 <= L <= 256.  The model and the oracle are defined for any L
 *     (Section 2.1), but the device recursion stores each vector only on the
 *     sublattice where it is nonzero, which needs a bipartite (even-L)
 *     periodic lattice; odd L is refused rather than run on a second, dense
 *     layout.  This departs from the reading that allows odd L on every path.
 *   b = 0 (a diagonal shift breaks that sublattice structure).
 *   M even, 2 <= M <= 8192; K a power of two with M <= K <= 8192 (the radix-2
 *     transform of the paper's node mapping runs in LDS).
 *   GFMC_FP32_ACC64 only inside its validated range (see gfmc_precision).
 */
#ifndef GFMC_H
#define GFMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GFMC_OK = 0,
  GFMC_EINVAL = -1,    /* invalid argument; state unchanged                  */
  GFMC_ENOMEM = -2,    /* workspace too small                                */
  GFMC_EDEVICE = -3,   /* HIP runtime error                                  */
  GFMC_EBUSY = -4,     /* resource busy                                      */
  GFMC_ESTATE = -5,    /* call not valid in the current state                */
  GFMC_ECANCELED = -6  /* operation cancelled                                */
} gfmc_status;

/* Precision of the Chebyshev recursion (Section 2.2, equation "recursive").
 * GFMC_FP64: FP64 throughout (moments within 1e-12, Delta S_eff within 1e-10
 * of the FP64 oracle).  GFMC_FP32_ACC64: vectors and stencil in FP32, the
 * moment sums (equation "mu2"), the reconstruction, the energy integral and
 * the acceptance in FP64.  Its rounding error grows with M and falls with L,
 * and the error of Delta S_eff grows with beta, so it is accepted only where
 * its measured error stays within 1e-5 on the moments and 2e-5 on Delta
 * S_eff: beta t <= 50 and M <= 1024 (L = 4, 6), 4096 (8 <= L < 16) or
 * 8192 (L >= 16); never on 2^3.  Elsewhere gfmc_workspace_bytes,
 * gfmc_chain_create, gfmc_set_params and gfmc_engine_submit return EINVAL,
 * unless params.fp32_unvalidated = 1 (for measuring that error). */
typedef enum { GFMC_FP64 = 0, GFMC_FP32_ACC64 = 1 } gfmc_precision;
typedef enum { GFMC_JACKSON = 0, GFMC_LORENTZ = 1 } gfmc_kernel;
typedef enum { GFMC_PROPOSE_SPHERE = 0, GFMC_PROPOSE_CONE = 1 } gfmc_proposal;
typedef enum { GFMC_INIT_RANDOM = 0, GFMC_INIT_FM = 1, GFMC_INIT_FM_PLUS_RANDOM = 2 } gfmc_init;
/* Start vectors of the recursion: the 7 unit vectors of o and its neighbours
 * (all 7x7 local moments), or the pair {|o>, |v> = Delta|o>} (only the three
 * series mu^{oo}, mu^{vv}, mu^{ov} that the 2x2 determinant needs; 2/7 of the
 * vector work per proposal), or the paper's mixed vectors {|o>, |v>, |o>+|v>,
 * |o>+i|v>} (Section 2.2: G_ov and G_vo formed from the diagonal Green's
 * functions of the mixed vectors).  On the bipartite lattice |o> and |v> never
 * share a sublattice at any step, so the mixed vectors' diagonal moments are
 * exact linear combinations of the pair's sums: GFMC_VECTORS_MIXED runs the
 * pair recursion and differs only in the reconstruction. */
typedef enum {
  GFMC_VECTORS_SITES = 0,
  GFMC_VECTORS_OV = 1,
  GFMC_VECTORS_MIXED = 2
} gfmc_vectors;
/* Hopping amplitudes in the Chebyshev step: recomputed from the per-site
 * spinor cache (16 B/site FP32), or read from a stored table of 6 amplitudes
 * per site (48 B/site FP32; the paper stores H in ELLPACK form).  Both give
 * bit-identical results; the stored form exists as an A/B measurement of the
 * matrix-free design and needs GFMC_VECTORS_SITES. */
typedef enum { GFMC_HOP_RECOMPUTE = 0, GFMC_HOP_STORED = 1 } gfmc_hoppings;

/* Parameters of one Markov chain (all energies in units of t). */
typedef struct {
  int32_t L;                /* linear size, N = L^3, periodic                         */
  double t;                 /* hopping scale (> 0)                                    */
  double beta;              /* inverse temperature (> 0)                              */
  double mu;                /* chemical potential                                     */
  int32_t M;                /* number of Chebyshev moments (even)                     */
  int32_t K;                /* energy nodes; 0 selects K = M                          */
  gfmc_kernel kernel;       /* damping kernel (Jackson default)                       */
  double lorentz_lambda;    /* Lorentz parameter; 0 selects 4.0                       */
  double scale_a;           /* Ht = (H - b)/a; 0 selects a = 6t/(1 - 0.01)            */
  double scale_b;           /* must be 0 on the device path                           */
  gfmc_precision precision; /* FP64, or FP32 recursion with FP64 moment sums          */
  gfmc_proposal proposal;   /* new direction: whole sphere or cap around the old one  */
  double cone_angle;        /* cap half-angle in rad (GFMC_PROPOSE_CONE)              */
  uint64_t seed;            /* Philox key word 0                                      */
  uint64_t chain_id;        /* Philox key word 1                                      */
  gfmc_vectors vectors;     /* start vectors (GFMC_VECTORS_SITES default)             */
  gfmc_hoppings hoppings;   /* hopping amplitudes (GFMC_HOP_RECOMPUTE default)        */
  int32_t fp32_unvalidated; /* 1: accept GFMC_FP32_ACC64 outside its validated range  */
                            /* (error measurements only; see GFMC_FP32_ACC64 below)   */
} gfmc_chain_params;

/* Outcome of one proposal (Algorithm 1, inner loop body). */
typedef struct {
  int64_t index;            /* proposal counter value sweep*N + j                     */
  int32_t site;             /* proposed site o                                        */
  int32_t own;              /* decision from (dseff, u): 1 accept                     */
  int32_t accepted;         /* decision applied (own unless forced)                   */
  int32_t pad_;
  double theta_old, phi_old, theta_new, phi_new;
  double dseff;             /* Delta S_eff = S_eff(new) - S_eff(old)                  */
  double u;                 /* uniform draw in [0,1) of the Metropolis test           */
  double phase_top;         /* continuous phase at the highest node (ideally ~0)      */
} gfmc_step_record;

typedef struct gfmc_chain gfmc_chain;   /* opaque */
typedef struct gfmc_batch gfmc_batch;   /* opaque */

/* ---------------------------------------------------------------- chains --
 * Device workspace (bytes, 256-byte aligned base) that a chain with these
 * parameters needs (the device-resident state of one Markov chain of
 * Algorithm 1, kept on the GPU across proposals as in Section 3, "Arrangement
 * of CUDA Kernel Functions"): spin angles, spinor cache, the 7 Chebyshev vectors (one
 * sublattice each, 7*N complex values), per-step moment partial sums, the
 * moment table and reconstruction scratch.  EINVAL for parameters outside the
 * device path's restrictions. */
gfmc_status gfmc_workspace_bytes(const gfmc_chain_params* params, size_t* bytes);

/* Create a chain on `dev_workspace` (device pointer of at least
 * gfmc_workspace_bytes bytes, owned by the caller, alive until destroy) and
 * `hip_stream` (hipStream_t, may be NULL for the default stream): one Markov
 * chain over the classical spins of the double-exchange model (Section 2.1;
 * Algorithm 1).  Spins start ferromagnetic (all theta = phi = 0); the
 * proposal counter starts at 0.  EINVAL for parameters outside the device
 * path's restrictions, ENOMEM if `bytes` is too small; on error *out is not
 * written and nothing is allocated.  destroy never frees the workspace. */
gfmc_status gfmc_chain_create(const gfmc_chain_params* params, void* dev_workspace,
                              size_t bytes, void* hip_stream, gfmc_chain** out);
gfmc_status gfmc_chain_destroy(gfmc_chain* chain);

/* Change the hopping scale t, the inverse temperature beta and the chemical
 * potential mu of the grand-canonical weight exp(-beta (H - mu N)) (Section
 * 2.1); the rescaling Ht = (H - b)/a of Section 2.2, if defaulted, follows t.
 * EINVAL (state unchanged) for non-positive t or beta, non-finite mu, or a
 * new (t, beta) outside the validated FP32 range of an FP32 chain. */
gfmc_status gfmc_set_params(gfmc_chain* chain, double t, double beta, double mu);

/* Initialise the classical spins (theta_i, phi_i) of Section 2.1 on the device
 * from the chain's Philox key: uniform on the sphere, ferromagnetic, or
 * ferromagnetic with exactly floor(frac*N) sites (picked by a partial
 * Fisher-Yates shuffle) redrawn on the sphere (the starting configuration of
 * Algorithm 1; the paper leaves it open).  EINVAL for an unknown mode or frac
 * outside [0, 1]. */
gfmc_status gfmc_init_spins(gfmc_chain* chain, gfmc_init mode, double random_fraction);

/* Copy the N spin angles (theta_i, phi_i) of equation "ht" from / to
 * caller-owned host arrays of N doubles each, site order i = x + L(y + Lz)
 * (theta in [0,pi], phi any finite value; EINVAL otherwise, state unchanged). */
gfmc_status gfmc_set_spins(gfmc_chain* chain, const double* theta, const double* phi);
gfmc_status gfmc_get_spins(gfmc_chain* chain, double* theta, double* phi);

/* Proposal counter (next proposal uses counter value `index`). */
gfmc_status gfmc_set_counter(gfmc_chain* chain, int64_t index);
gfmc_status gfmc_get_counter(gfmc_chain* chain, int64_t* index);

/* Failure detection.  Number of the chain's proposals whose Delta S_eff
 * (eq. "d_seff2") came out non-finite since creation: each was rejected,
 * whatever a forced decision said, and left the chain unchanged.  A growing
 * count means the chain's state is corrupted (e.g. non-finite angles written
 * into its workspace); other chains of a batch are unaffected.  Waits for the
 * chain's stream.  EINVAL for NULL arguments. */
gfmc_status gfmc_chain_nonfinite(gfmc_chain* chain, int64_t* count);

/* Device addresses of the chain's spin angles theta, phi (N doubles each,
 * site order as gfmc_set_spins) inside its caller-owned workspace, for reading
 * them without a copy to the host.  Values written there bypass
 * gfmc_set_spins's validation and the spinor cache (which gfmc_set_spins
 * rebuilds); the library reads them when it forms a proposal's bond changes.
 * EINVAL for NULL arguments. */
gfmc_status gfmc_chain_device_angles(gfmc_chain* chain, double** theta, double** phi);

/* Local moments mu_n^{jk} = <j|T_n(Ht)|k>, n < M, around `site` for the current
 * spins (no state change): the Chebyshev moments of Section 2.2 from M/2 steps
 * of the recursion (equation "recursive") with doubling (equation "mu2"),
 * start vectors j, k over `site` and its six neighbours.  Writes
 * mu[M][7][7][2] (caller-owned host array, FP64, re/im).  EINVAL for a site
 * outside [0, N) or mu NULL; ESTATE for chains not created with
 * GFMC_VECTORS_SITES. */
gfmc_status gfmc_moments(gfmc_chain* chain, int32_t site, double* mu);

/* Moments of the pair {|o>, |v>} for moving the spin at `site` to
 * (theta_new, phi_new), no state change: mu[n][s][2] with s = 0: <o|T_n|o>,
 * 1: <v|T_n|v>, 2: <o|T_n|v>, |v> = sum_d Delta_{n_d,o} |n_d>.  Chains created
 * with GFMC_VECTORS_OV or GFMC_VECTORS_MIXED only (ESTATE otherwise). */
gfmc_status gfmc_pair_moments(gfmc_chain* chain, int32_t site, double theta_new, double phi_new,
                              double* mu);

/* Diagonal moments of the paper's mixed start vectors (Section 2.2) for moving
 * the spin at `site` to (theta_new, phi_new), no state change: mu[s][n] (host,
 * real, 4*M values) = <a_s|T_n(Ht)|a_s> with a_0 = |o>, a_1 = |v>,
 * a_2 = |o>+|v>, a_3 = |o>+i|v>, |v> = sum_d Delta_{n_d,o} |n_d>.  Chains
 * created with GFMC_VECTORS_OV or GFMC_VECTORS_MIXED only (ESTATE otherwise). */
gfmc_status gfmc_mixed_moments(gfmc_chain* chain, int32_t site, double theta_new,
                               double phi_new, double* mu);

/* Delta S_eff = S_eff(new) - S_eff(old) for moving the spin at `site` to
 * (theta_new, phi_new), no state change: the kernel-damped local Green's
 * functions (equations "green", "green_short", "green_fft"), the 2x2
 * determinant d(z) of equation "d_z_green" and the Fermi-weighted phase
 * integral of equation "d_seff2".  *dseff (host) receives the value;
 * phase_top (may be NULL) the continuous phase of d at the highest node
 * (ideally ~0).  EINVAL for a site outside [0, N), non-finite angles or
 * dseff NULL. */
gfmc_status gfmc_delta_seff(gfmc_chain* chain, int32_t site, double theta_new,
                            double phi_new, double* dseff, double* phase_top);

/* One proposal at the chain's counter: the body of Algorithm 1's inner loop
 * (random site and direction, Delta from equation "ht", Delta S_eff, the
 * Metropolis test e^{-Delta S} > u, spin update).  force -1 takes the
 * chain's own decision, 0 rejects, 1 accepts (teacher forcing for parity
 * runs).  rec (host, may be NULL) receives the record.  EINVAL for force
 * outside -1..1. */
gfmc_status gfmc_step(gfmc_chain* chain, int32_t force, gfmc_step_record* rec);

/* nsweeps sweeps of N proposals each (Algorithm 1, outer loop), with the
 * magnetization |sum_i S_i| / N after each sweep (Algorithm 1, after the
 * inner loop).  magnetization [nsweeps] and accepted (total over the call)
 * are caller-owned host arrays and may be NULL.  EINVAL for nsweeps < 0. */
gfmc_status gfmc_sweep(gfmc_chain* chain, int32_t nsweeps, double* magnetization,
                       int64_t* accepted);

/* The magnetization |sum_i S_i| / N of the chain's current spins, S_i the unit
 * vector of (theta_i, phi_i) (Algorithm 1, the measurement after each sweep),
 * computed on the device; *m (host) receives it.  EINVAL for m NULL. */
gfmc_status gfmc_magnetization(gfmc_chain* chain, double* m);

/* Wait for the chain's enqueued device work (its stream). */
gfmc_status gfmc_sync(gfmc_chain* chain);

/* ----------------------------------------------------------------- batches --
 * A batch advances several independent chains together: every Chebyshev step
 * is one launch over all chains that still need it, so chains of different L
 * and M share the device.  All chains must have the same precision and be
 * created on the same device; the batch enqueues on its own stream and the
 * chains must not be used individually while the batch exists.
 * The batch workspace holds the chain descriptor table and launch plans. */
gfmc_status gfmc_batch_workspace_bytes(gfmc_chain* const* chains, int32_t n, size_t* bytes);
gfmc_status gfmc_batch_create(gfmc_chain* const* chains, int32_t n, void* dev_workspace,
                              size_t bytes, void* hip_stream, gfmc_batch** out);
gfmc_status gfmc_batch_destroy(gfmc_batch* batch);

/* nprop proposals on every chain.  force: NULL (own decisions) or [nprop][n];
 * recs: NULL or [nprop][n] records. */
gfmc_status gfmc_batch_step(gfmc_batch* batch, int32_t nprop, const int32_t* force,
                            gfmc_step_record* recs);

/* Each chain runs nsweeps sweeps of its own N proposals; magnetization
 * [n][nsweeps] and accepted [n] may be NULL.  Chains with smaller N finish
 * their sweeps earlier and stop. */
gfmc_status gfmc_batch_sweep(gfmc_batch* batch, int32_t nsweeps, double* magnetization,
                             int64_t* accepted);

/* Capture one proposal of the whole batch (propose, every Chebyshev step,
 * moment assembly, reconstruction and Metropolis update) in a HIP graph and
 * replay it for later gfmc_batch_step calls without force or records
 * (enable != 0), or go back to direct launches (enable == 0). */
gfmc_status gfmc_batch_use_graph(gfmc_batch* batch, int32_t enable);

/* Launch shape of the Chebyshev steps: 1 or 2 site pairs per thread of the
 * multi-block step kernel (one launch per step; with 2, the pair form and the
 * FP32 7-vector form take the two pairs from one y column of a z-plane and
 * share their y neighbours' loads), or 0 for one LDS-resident
 * workgroup per chain that runs all M/2 steps in a single launch (every
 * chain must fit: 128 B/site FP32, 232 B/site FP64 within 140 KB, i.e. up
 * to 10^3 FP32 / 8^3 FP64, 7 site start vectors, recomputed hoppings).
 * Shape 3 (pair form only, GFMC_VECTORS_OV or GFMC_VECTORS_MIXED, with
 * recomputed hoppings): step 1 as shape 1, then two Chebyshev steps per
 * launch, each block advancing a tile of full x-rows staged in LDS with two
 * halo rows in y and z (Section 2.2's three series need only the pair of
 * vectors, so a tile of both slots and the spinors fits); needs L >= 8
 * divisible by the tile rows (8, 4 or 2, FP32 up to L = 64 and FP64 up to
 * L = 32 with the 144 KB tile), lock-step proposals (EINVAL in the
 * step-granular schedule) and uses one step lane.  Vector values agree bit
 * for bit with shape 1.  Results do not depend on the shape beyond the order
 * of the moment partial sums.  Single chains, and new batches whose chains
 * all fit, use shape 0; otherwise shape 1.  EINVAL when a chain does not fit
 * the shape asked for. */
gfmc_status gfmc_batch_set_tuning(gfmc_batch* batch, int32_t pairs_per_thread);

/* Step lanes: 1 (every Chebyshev step one launch on the batch stream) to 4
 * (the chains, in plan order, split into that many ranges of about equal work
 * whose steps run on streams owned by the batch, forked from the batch stream
 * before the steps of a proposal and joined back after them; the launches of
 * one range fill the ramp-up and tail of the others').  Work stays ordered on
 * the batch stream; per-chain results do not depend on the lanes.  Lanes need
 * a multi-block shape (1 or 2) and at most one lane per chain is used.
 * EINVAL outside 1..4. */
gfmc_status gfmc_batch_set_lanes(gfmc_batch* batch, int32_t lanes);

/* Schedule of gfmc_batch_step over chains of different step counts M/2
 * (independent Markov chains, Section 3 "Parallelization Frameworks";
 * Algorithm 1 per chain).  0 (default), lock-step: every chain makes exactly
 * nprop proposals and a chain with fewer steps idles until the longest
 * chain's proposal ends.  1, step-granular: the chains with the most steps
 * make nprop proposals in nprop x M_max/2 step rounds, and every other chain
 * makes as many whole proposals as fit in those rounds, floor(nprop x
 * M_max / M), each started right after the reconstruction of its last, so a
 * chain of half the steps makes twice the proposals.  Chains of equal M (per
 * step lane) draw, step and reconstruct together; every Chebyshev step of
 * the others runs in one launch per round (per lane) that reads each
 * chain's step index from the round.  Per-chain results equal the lock-step
 * ones proposal for proposal.  Step-granular batches take no force or
 * records (EINVAL); gfmc_batch_sweep always runs lock-step; the LDS-resident
 * shape (one launch per proposal) is unaffected.  EINVAL outside {0, 1}. */
gfmc_status gfmc_batch_set_schedule(gfmc_batch* batch, int32_t step_granular);

/* Non-temporal memory access in the Chebyshev steps of the 7-vector
 * multi-block kernel (on != 0): each site's own a_{s-2} is loaded and a_s
 * stored without retaining the lines in the caches.  Pays where a batch's
 * vectors stream from HBM (working sets well above the 256 MB last-level
 * cache); slower where they fit it.  Results do not depend on it.
 * gfmc_batch_autotune chooses it with the launch shape.  EINVAL outside
 * {0, 1}. */
gfmc_status gfmc_batch_set_nontemporal(gfmc_batch* batch, int32_t on);

/* Threads per block of the launched Chebyshev step kernel (launch shapes 1
 * and 2; the LDS-resident and persistent kernels have block sizes of their
 * own): 256 (default) or, for the 7-vector form with recomputed hoppings,
 * 512.  The block partial sums of the moments then group the sites
 * differently (results agree to rounding of the FP64 sums; the vectors bit
 * for bit).  gfmc_batch_autotune chooses it with the launch shape.  EINVAL
 * for other values, or 512 with the pair or mixed start vectors or stored
 * hoppings. */
gfmc_status gfmc_batch_set_block_threads(gfmc_batch* batch, int32_t threads);
gfmc_status gfmc_batch_get_block_threads(gfmc_batch* batch, int32_t* threads);

/* Execution form in effect: *resident = 1 when every chain runs all its
 * steps in one LDS-resident workgroup; *persistent = the number of working
 * blocks when a lone chain runs all its steps in one persistent launch on
 * one compute die (0 otherwise); *step_granular = the schedule set by
 * gfmc_batch_set_schedule; *nontemporal = gfmc_batch_set_nontemporal's
 * setting.  Pointers may be NULL. */
gfmc_status gfmc_batch_get_form(gfmc_batch* batch, int32_t* resident, int32_t* persistent,
                                int32_t* step_granular, int32_t* nontemporal);

/* Launch shape (0 to 3) and number of step lanes in effect. */
gfmc_status gfmc_batch_get_tuning(gfmc_batch* batch, int32_t* pairs_per_thread, int32_t* lanes);

/* Time each step-kernel launch shape the batch's chains fit (shape 3 only
 * in the lock-step schedule; non-temporal access and 512-thread blocks for
 * the 7-vector kernel; for a lone chain that fits one die, its persistent
 * kernel) with one to
 * four lanes over max(trial_steps, 64) Chebyshev steps (at most M/2 - 1) on
 * the batch's current spins (no change of chain state), by host wall time
 * (so that the host's launch rate counts where launches are short), keep
 * the fastest, and remember it for later batches of the same shape
 * (precision, start vectors, hoppings, schedule, number of chains, L and M
 * of each chain).  chosen (the shape) may be NULL; gfmc_batch_get_tuning
 * reports the lanes. */
gfmc_status gfmc_batch_autotune(gfmc_batch* batch, int32_t trial_steps, int32_t* chosen);

/* Timing of the Chebyshev step kernel over the last gfmc_batch_step call,
 * from HIP events on the batch stream around the step launches: total
 * milliseconds and number of step rounds (one round = one step of every
 * chain still stepping: one launch, or one per lane). */
gfmc_status gfmc_batch_step_timing(gfmc_batch* batch, double* step_ms, int64_t* launches);

/* Algorithmic bytes moved by one proposal of `chain` in the step kernel
 * (vectors read and written, spinors read; per step and summed over steps). */
gfmc_status gfmc_chain_step_bytes(gfmc_chain* chain, double* bytes_per_step, int32_t* steps);

/* ----------------------------------------------------------------- serving --
 * An engine runs independent chain requests on one device with continuous
 * batching: a host worker thread admits queued requests whenever a slot and
 * enough of the HBM budget are free (in arrival order; a request whose
 * workspace does not fit yet lets later ones that fit go first, until it has
 * waited 10 s, after which the requests behind it wait for it), and every
 * iteration advances all
 * admitted chains by one proposal in one batched launch sequence, so chains
 * of different L, M and temperature share the device and requests that
 * arrive while others run join at the next iteration.  Each request runs
 * `nsweeps` sweeps (N proposals each, Algorithm 1) from its own Philox key
 * and start configuration; per-chain results do not depend on which other
 * chains share the device.  The engine owns one device allocation of
 * `hbm_budget_bytes` (chain workspaces are carved from it) and one stream. */
typedef struct gfmc_engine gfmc_engine;   /* opaque */

typedef struct {
  uint64_t request_id;
  gfmc_status status;       /* GFMC_OK, GFMC_ECANCELED, or the error that stopped it  */
  int32_t L, M;
  int32_t sweeps;           /* completed sweeps                                       */
  int32_t pad_;
  int64_t proposals, accepted;
  double magnetization;     /* |m| after the last completed sweep                     */
  double magnetization_mean;/* mean of |m| over completed sweeps                      */
  double t_submit, t_admit, t_first_sweep, t_done;   /* seconds since engine creation */
} gfmc_result;

gfmc_status gfmc_engine_create(int device, size_t hbm_budget_bytes, int32_t max_slots,
                               gfmc_engine** out);
/* Queue a request.  EBUSY if its workspace alone exceeds the engine's budget
 * (it could never be admitted); EINVAL for invalid parameters or nsweeps < 1. */
gfmc_status gfmc_engine_submit(gfmc_engine* engine, const gfmc_chain_params* params,
                               gfmc_init init, double random_fraction, int32_t nsweeps,
                               uint64_t* request_id);
/* Move up to `cap` finished results into `out`; *n receives how many. */
gfmc_status gfmc_engine_poll(gfmc_engine* engine, gfmc_result* out, int32_t cap, int32_t* n);
/* Cancel a queued or running request (its result reports GFMC_ECANCELED);
 * EINVAL if the id is unknown or already finished. */
gfmc_status gfmc_engine_cancel(gfmc_engine* engine, uint64_t request_id);
/* Drain the recorded wall-clock durations (seconds) of completed sweeps, in
 * completion order, and the matching request ids (ids may be NULL). */
gfmc_status gfmc_engine_sweep_latencies(gfmc_engine* engine, double* seconds, uint64_t* ids,
                                        int32_t cap, int32_t* n);
/* Counts: queued, running, finished-but-unpolled requests; bytes in use. */
gfmc_status gfmc_engine_status(gfmc_engine* engine, int32_t* queued, int32_t* running,
                               int32_t* finished, size_t* bytes_in_use);
/* Block until no request is queued or running (or timeout_s elapses: EBUSY). */
gfmc_status gfmc_engine_drain(gfmc_engine* engine, double timeout_s);
/* Stop the worker (running requests are cancelled) and free the device memory. */
gfmc_status gfmc_engine_destroy(gfmc_engine* engine);

/* ----------------------------------------------------- allocation-free --
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Delta S_eff
 * as gfmc_delta_seff computes it, with the kernels and launch shape of such a
 * chain in a batch (the LDS-resident kernel where it fits, else one step
 * launch per Chebyshev step: the same value bit for bit as gfmc_delta_seff
 * where that takes the same shape; on a lone multi-block chain small enough
 * for one compute die gfmc_delta_seff runs the persistent kernel, whose block
 * sums group the sites differently, and the two agree to rounding of the FP64
 * sums), for the spins in the caller's device arrays d_theta[N] and
 * d_phi[N] (FP64, read only) and the move of `site` to (theta_new, phi_new),
 * with no chain handle and no workspace.  Every intermediate buffer lives in
 * a static device array of the library, 64 MiB per device, held from the
 * first use of the library on that device until the process ends; no call
 * allocates or frees device memory.  Parameters whose buffers exceed 64 MiB
 * (e.g. 32^3 with M above 2048, 64^3) return EINVAL.  All work is enqueued on
 * `hip_stream` (NULL: the default stream); *d_dseff and, if non-NULL,
 * *d_phase_top are device doubles written by the last kernel.  The array is
 * shared by every call on a device: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller. */
gfmc_status gfmc_delta_seff_static(const gfmc_chain_params* params, const double* d_theta,
                                   const double* d_phi, int32_t site, double theta_new,
                                   double phi_new, double* d_dseff, double* d_phase_top,
                                   void* hip_stream);

/* ------------------------------------------------------------ calibration --
 * Streaming bandwidth of the device, the practical ceiling against which the
 * step kernel's algorithmic bandwidth is read (no paper passage: measurement
 * infrastructure).  mode 0 reads `a`, 1 writes `c`, 2 copies `a` to `c`,
 * 3 writes a + b to `c` (two reads per write, the step kernel's mix); each
 * buffer is a caller-owned device allocation of `bytes` (a multiple of 16;
 * `c` is always required, 16 bytes suffice in mode 0).  For grids of 2, 4, 8
 * and 16 blocks per compute unit: one warm-up pass, then `reps` timed passes
 * on `stream`; *gbs = the best of bytes moved once per pass (1, 1, 2 or 3
 * buffers) x reps / elapsed time, in GB/s.  Buffers well above the 256 MB
 * last-level cache measure HBM; smaller ones the cache. */
gfmc_status gfmc_stream_bandwidth(int32_t mode, const void* a, const void* b, void* c,
                                  size_t bytes, int32_t reps, void* stream, double* gbs);

/* ------------------------------------------------------------------ misc -- */
const char* gfmc_status_string(int32_t status);   /* any value: unknown ones named so */
const char* gfmc_last_error(void);
const char* gfmc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GFMC_H */
