// gfmc_device.h -- device-side data layout and small helpers of the gfx950
// GFMC library.  Included only by the library's own translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfmc.h"

namespace gfmc {

constexpr int kStepThreads = 256;   // threads per block of the Chebyshev step kernel
constexpr int kStepWaves = kStepThreads / 64;
// The persistent lone-chain kernel runs blocks of 64, 128 or 256 threads, at
// most one per compute unit of one die.
constexpr int kPersistMaxBlocks = 32;
constexpr int kResThreads = 1024;   // threads of the LDS-resident workgroup (4 waves per SIMD)
constexpr int kNP = 49;             // moment partial sums per block and step (7 site vectors)
constexpr int kNP2 = 4;             // ... for the pair {o, v}
constexpr int kReconThreads = 256;  // threads of the reconstruction block (one per chain)
constexpr int kRecCap = 64;         // proposals per host round trip (records, forcing)
constexpr int kMagCap = 64;         // sweeps per host round trip (magnetization)
constexpr int kMaxK = 8192;         // energy nodes held in LDS by the transform
// dynamic LDS of the single-workgroup (LDS-resident) Chebyshev kernel; the
// kernel's static LDS (staging and Gram sums) is 16.9 KB of the 160 KB
constexpr int kResidentLds = 140 * 1024;
// two-step pair-form kernel: threads per block (one tile) and the most
// dynamic LDS a tile may take
constexpr int kTileThreads = 1024;
constexpr int kTileLds = 144 * 1024;

// Complex value and per-site spinor in the recursion precision T.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};
template <typename T>
struct alignas(16) spn {   // chi = (alpha, beta) = (cos(th/2) e^{-i ph/2}, sin(th/2) e^{i ph/2})
  T ar, ai, br, bi;
};

// Per-chain control block (device).  Written by the proposal and
// reconstruction kernels, read by the Chebyshev steps.
struct Ctl {
  int64_t index;            // counter value of the next proposal
  int64_t accepted_total;   // accepted proposals since creation
  int64_t nonfinite;        // proposals whose Delta S_eff was not finite (rejected)
  int32_t mode;             // 0 draw from the counter, 1 host-given site+angles, 2 site only
  int32_t site;             // proposed site o
  int32_t parity_o;         // (x+y+z) & 1 of o
  int32_t o_half;           // half-row index of o
  int32_t start_site[7];    // o and its neighbours, full site index
  int32_t start_half[7];    // ... half-row index
  int32_t own, accepted;
  double th_old, ph_old, th_new, ph_new, u, dseff, phase_top;
  double delta[12];         // Delta_{n_d,o}, d = 0..5 (re, im)
  // persistent single-chain step kernel, cleared by the proposal kernel:
  // [0] tickets handed out, [1] 1 + the compute die (XCD) that claimed the
  // run, [2] barrier arrivals, [3] nonzero when a barrier wait timed out
  unsigned bar[4];
};

// Division by a per-chain constant d for 0 <= n < 2^31: m = floor((2^32 - 1)
// / d) makes the high word of n m undershoot n / d by at most one, which one
// comparison corrects (the step kernels split every site index this way
// instead of by a division instruction sequence).
struct FastDiv {
  uint32_t d, m;
};
__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
  return FastDiv{d, (uint32_t)(0xffffffffu / d)};
}

// Per-chain descriptor (device table read by the batched kernels).
struct Desc {
  int32_t L, N, half, M, S, K, nblk, kernel, proposal, log2K;
  int32_t vectors, hops;      // GFMC_VECTORS_*, GFMC_HOP_*
  int32_t tile_y, tile_z;    // two-step pair kernel: rows per tile in y and z
  FastDiv div_hx, div_L;     // division by L/2 and by L (site index splitting)
  double t, beta, mu, a, cone, lambda;
  uint64_t seed, chain_id;
  double* theta;            // [N]
  double* phi;              // [N]
  void* spin;               // spn<T>[2][half]   (parity, half-row index)
  void* vec;                // o-slots cpx<T>[2][half], then n-slots: six values per
                            // [2][half] entry as 16-byte planes (3 FP32 / 6 FP64)
                            // ({o,v}: o-slots, then v-slots cpx<T>[2][half])
  double* part;             // [S][nblk][kNP] ({o,v}: [S][nblk][kNP2])
  double* mom;              // [M][7][7][2]  ({o,v}: [M][3][2])
  double* gscr;             // [4][K][2]
  void* hop;                // GFMC_HOP_STORED: t_{i, n_d(i)}, [2][half] entries,
                            // same plane layout as the n-slots
  double* tab;              // per-chain constant tables of the reconstruction:
                            // g[M], pre[K][2], tw[K/2][2], sinth[K], wt[K]
  Ctl* ctl;
};

// Tiles of the two-step pair-form kernel: ty x tz full x-rows of one chain,
// staged in LDS with two halo rows on each side in y and z (o-slot, v-slot
// and spinor of every site: 32 B in FP32, 64 B in FP64).  The largest of
// 8x8, 8x4, 4x4, 4x2, 2x2 that divides L and fits kTileLds; false if none.
__host__ __device__ inline bool tile_dims(int L, int fp32, int* ty, int* tz) {
  const int bytes = fp32 ? 32 : 64;
  const int cand[5][2] = {{8, 8}, {8, 4}, {4, 4}, {4, 2}, {2, 2}};
  for (int i = 0; i < 5; ++i) {
    const int y = cand[i][0], z = cand[i][1];
    if (L % y != 0 || L % z != 0) continue;
    if ((long long)(y + 4) * (z + 4) * L * bytes <= kTileLds) {
      *ty = y;
      *tz = z;
      return true;
    }
  }
  return false;
}

// Site decomposition of the bipartite layout: site (x,y,z) has parity
// (x+y+z)&1 and half-row index (x>>1) + (L/2)(y + L z); the two sites of a
// given half-row index differ only in the low bit of x.
__host__ __device__ inline int half_index(int x, int y, int z, int L) {
  return (x >> 1) + (L >> 1) * (y + L * z);
}

}  // namespace gfmc
