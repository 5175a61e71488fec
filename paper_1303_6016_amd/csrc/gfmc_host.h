// gfmc_host.h -- host-side internals shared by the C ABI translation units
// (chain/batch handles, workspace layout, launch plans).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "gfmc_device.h"

namespace gfmc {
hipError_t launch_propose(const Desc* d, int n, hipStream_t st);
// One Chebyshev step launch over chains [0, nact) of table d.  act_end NULL:
// every chain takes step s.  act_end non-NULL: s is the round of a window and
// chain c takes step (s - 1) mod S_c + 1 while s <= act_end[c] (never step 1).
// nt: non-temporal loads of each site's own a_{s-2} and stores of a_s (steps >= 2
// of the 7-vector kernel; pays where the batch streams from HBM).
// bt: threads per block of the step kernel (kStepThreads, or 512 for the
// 7-vector form with recomputed hoppings).
hipError_t launch_step(int fp32, int ov, int hops, int ppt, const Desc* d, const int* blkoff,
                       int nact, int blocks, int s, hipStream_t st, const int* act_end = nullptr,
                       int nt = 0, int bt = kStepThreads);
hipError_t prepare_step_ov2();
hipError_t launch_step_ov2(int fp32, const Desc* d, const int* tileoff, int nact, int tiles, int s,
                           size_t lds, hipStream_t st);
hipError_t launch_moments(int ov, const Desc* d, int n, int smax, hipStream_t st);
hipError_t launch_recon(int fp32, const Desc* d, int n, int kmax, const int32_t* force,
                        gfmc_step_record* recs, hipStream_t st);
hipError_t launch_spinors(int fp32, const Desc* d, int n, int nmax, hipStream_t st);
hipError_t launch_hops(int fp32, const Desc* d, int nmax, hipStream_t st);
hipError_t launch_resident(int fp32, const Desc* d, int n, size_t lds, hipStream_t st);
// Persistent single-chain step run (cooperative launch of 8 nb blocks, nb work).
hipError_t launch_persist(int fp32, const Desc* d, int nb, int threads, hipStream_t st);
// counts[die] (16 unsigned, zeroed by the caller) += blocks landing on each die.
hipError_t launch_die_census(unsigned* counts, int blocks, hipStream_t st);
hipError_t launch_init_spins(const Desc* d, int nmax, int mode, hipStream_t st);
hipError_t launch_fisher_yates(const Desc* d, int64_t nr, int32_t* perm, hipStream_t st);
hipError_t launch_magnetization(const Desc* d, int n, double* out, hipStream_t st);
hipError_t launch_tables(const Desc* d, int kmax, hipStream_t st);
hipError_t launch_mixed_series(const Desc* d, int M, double* out, hipStream_t st);
}  // namespace gfmc

using namespace gfmc;

gfmc_status gfmc_fail(gfmc_status s, const std::string& msg);

// Enum-typed arguments and fields arrive from C callers and language bindings
// as 32-bit integers of any value; they are validated as integers, read from
// their bytes, before anything reads them as their enum type.
template <typename E>
inline int32_t gfmc_enum_value(const E& v) {
  static_assert(sizeof(E) == sizeof(int32_t), "enums of the C ABI are 32-bit");
  int32_t r;
  std::memcpy(&r, &v, sizeof r);
  return r;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return gfmc_fail(GFMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

#define CHK(expr)                          \
  do {                                     \
    gfmc_status s_ = (expr);               \
    if (s_ != GFMC_OK) return s_;          \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kMaxLanes = 4;   // step lanes (streams) of a batch
constexpr int kShapeTile2 = 3;  // launch shape: pair form, two Chebyshev steps per launch

// ------------------------------------------------------- chain layout ----
struct Derived {
  int L, N, half, M, S, K, log2K, nblk, fp32, ov, hops;
  int part_blocks;   // partial-sum slots per step (the most blocks of any step form)
  double a, lambda;
};

struct Layout {
  size_t desc, blkoff, force, rec, mag, ctl, theta, phi, spin, hop, vec, part, mom, gscr, tab,
      total;
};

// A launch plan: a device table of chain descriptors (sorted by number of
// Chebyshev steps, largest first) and the block offsets of the step kernel.
struct Plan {
  int n = 0, fp32 = 0, smax = 0, kmax = 0, nmax = 0;
  int nt = 0;                          // non-temporal own loads and stores in the steps
  int ppt = 1;                         // site pairs per thread of the step kernel;
                                       // 0: one LDS-resident workgroup per chain;
                                       // kShapeTile2: pair form, two steps per launch
                                       // (step 1 and the partial sums as with 1)
  std::vector<int> tileoff;            // kShapeTile2: tile offsets per sorted chain (n + 1)
  int* d_tileoff = nullptr;            // ... device copy (batches only)
  size_t tile_lds = 0;                 // kShapeTile2: dynamic LDS of the launches
  int resident = 0;                    // shape 0 in effect (every chain fits in LDS)
  int persist = 0;                     // > 0: a lone chain's steps in one launch of this
                                       // many working blocks on one die (persistent kernel);
                                       // < 0: candidate, pending the die census
  bool allow_persist = false;          // chain and batch plans (not the engine's groups)
  Ctl* persist_ctl = nullptr;          // the lone chain's control block (timeout flag)
  int persist_threads = 0;             // threads per block of the persistent kernel
  int step_threads = kStepThreads;     // threads per block of the launched step kernel
  size_t res_lds = 0;                  // dynamic LDS of the resident kernel
  int ov = 0;                          // start vectors {o, v} instead of the 7 sites
  int hops = 0;                        // stored hopping table instead of recompute
  Desc* d_desc = nullptr;
  int* d_blkoff = nullptr;
  int32_t* d_force = nullptr;          // [kRecCap][n]
  gfmc_step_record* d_rec = nullptr;   // [kRecCap][n]
  double* d_mag = nullptr;             // [kMagCap][n]
  std::vector<int> S, blkoff;          // per sorted chain; blkoff has n+1 entries
  hipStream_t stream = nullptr;
  // Step lanes: with lanes = k >= 2 the sorted chains are split into k
  // contiguous ranges of about equal work whose Chebyshev steps run on k
  // streams of the plan, forked from `stream` before the steps and joined
  // back after them, so that one range's launches fill the ramp-up and tail
  // of the others'.  Everything else of a proposal stays on `stream`.
  int lanes = 1;                       // requested: 1 .. kMaxLanes
  int lanes_on = 1;                    // in effect (<= number of chains; 1 for shape 0)
  int lane_first[kMaxLanes] = {}, lane_n[kMaxLanes] = {};
  std::vector<int> lane_blkoff[kMaxLanes];   // block offsets within each lane (lane_n + 1)
  int* d_lane_blkoff[kMaxLanes] = {};
  hipStream_t lane_stream[kMaxLanes] = {};  // created on first use, owned
  hipEvent_t fork = nullptr, join[kMaxLanes] = {};
  // timing of the step launches
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  double step_ms = 0;
  int64_t step_launches = 0;
  bool timing = false;
  // graph replay of one proposal
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // Step-granular schedule (cont = 1): within a window each chain runs its
  // proposals back to back, a chain of S steps starting its next proposal
  // right after the step rounds of its last, so chains with fewer steps make
  // more proposals while longer ones keep stepping.  A cohort is a run of
  // chains of one lane with equal S: they start, finish and reconstruct
  // together.  act_end[c] is chain c's last active round of the window.
  int cont = 0;
  struct Cohort {
    int lane = 0, first = 0, n = 0, S = 0, kmax = 0;
    std::vector<int> blkoff;            // n + 1 block offsets within the cohort
    int* d_blkoff = nullptr;
  };
  std::vector<Cohort> coh;
  int* d_coh_blkoff = nullptr;          // device region of 2 n + 8 ints (cohort tables)
  int* d_act_end = nullptr;             // device [n], plan order
  std::vector<int> act_end;             // host copy of what the device holds
};

struct gfmc_chain {
  gfmc_chain_params p;
  Derived d;
  Layout l;
  char* ws = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  Desc desc;
  Plan plan;            // single-chain plan living in the chain's workspace
  bool in_batch = false;
};

struct gfmc_batch {
  std::vector<gfmc_chain*> chains;   // caller order
  std::vector<gfmc_chain*> sorted;   // plan order
  std::vector<int> order;            // sorted position -> caller index
  Plan plan;
  bool use_graph = false;
};


gfmc_status derive(const gfmc_chain_params* p, Derived& d);
bool resident_fits(const Derived& d);   // the LDS-resident kernel can hold the chain
bool resident_ok(const Derived& d);     // ... and is the preferred shape for it
Layout layout_of(const Derived& d);
void fill_desc(gfmc_chain* c);
gfmc_status upload_plan(Plan& P, const std::vector<gfmc_chain*>& sorted);
void plan_shape(Plan& P, const std::vector<gfmc_chain*>& sorted);
gfmc_status enqueue_steps(Plan& P, int s_first, int s_last);
void release_lanes(Plan& P);
gfmc_status enqueue_proposal(Plan& P, const int32_t* d_force, gfmc_step_record* d_rec,
                             bool with_recon);
// After proposals that used the persistent kernel: EDEVICE if one of its
// barrier waits timed out (that proposal left the chain unchanged; the plan
// falls back to one launch per step).
gfmc_status persist_check(Plan& P);
// Step-granular window of `rounds` step rounds (cont = 1): chain c runs
// min(rounds / S_c, cap[c]) whole proposals (cap NULL: no cap) and
// props[c] (plan order, may be NULL) receives that count.
// enqueue = false only computes the counts and uploads act_end (before a capture).
gfmc_status enqueue_window(Plan& P, int rounds, const int* cap, int* props, bool enqueue = true);
gfmc_status chain_setup(gfmc_chain* c, const gfmc_chain_params* p, const Derived& d, void* ws,
                        size_t bytes, hipStream_t stream);
gfmc_status chain_init_spins(gfmc_chain* c, int mode, double frac);
