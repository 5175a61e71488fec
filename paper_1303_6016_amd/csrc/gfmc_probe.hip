// gfmc_probe.hip -- streaming-bandwidth calibration of the device (the
// ceiling the step kernel's algorithmic bandwidth is compared against).
//
// Four access patterns over caller buffers of `bytes` each, 16-byte items,
// grid-stride with one item per thread and pass (measured on MI355X: four
// independent items per thread in flight, spread a grid apart, stream 10-20 %
// slower from HBM): read only, write only, copy (one read + one write), and
// two reads + one write (the step kernel's mix of stored values read to
// values written is 2 : 1).  Grids of 2 to 16 blocks per compute unit are
// timed and the fastest counts.  The rate counts the bytes each pattern must
// move once: 1, 1, 2 and 3 buffers per pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "gfmc_host.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kUnroll = 1;

template <int MODE>
__global__ __launch_bounds__(256) void k_stream(const f4* __restrict__ a, const f4* __restrict__ b,
                                                f4* __restrict__ c, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    f4 va[kUnroll], vb[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (MODE != 1) va[u] = a[i + u * stride];
      if (MODE == 3) vb[u] = b[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (MODE == 0) acc += va[u];
      else if (MODE == 1) c[i + u * stride] = f4{1.f, 2.f, 3.f, 4.f};
      else if (MODE == 2) c[i + u * stride] = va[u];
      else c[i + u * stride] = va[u] + vb[u];
    }
  }
  for (; i < n; i += stride) {
    if (MODE == 0) acc += a[i];
    else if (MODE == 1) c[i] = f4{1.f, 2.f, 3.f, 4.f};
    else if (MODE == 2) c[i] = a[i];
    else c[i] = a[i] + b[i];
  }
  // keeps the reads of the read-only pattern (never true for finite data)
  if (MODE == 0 && acc.x != acc.x) c[0] = acc;
}

template <int MODE>
hipError_t launch(const f4* a, const f4* b, f4* c, size_t n, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_stream<MODE>, dim3(grid), dim3(256), 0, st, a, b, c, n);
  return hipGetLastError();
}

hipError_t launch_mode(int mode, const f4* a, const f4* b, f4* c, size_t n, int grid,
                       hipStream_t st) {
  switch (mode) {
    case 0: return launch<0>(a, b, c, n, grid, st);
    case 1: return launch<1>(a, b, c, n, grid, st);
    case 2: return launch<2>(a, b, c, n, grid, st);
    default: return launch<3>(a, b, c, n, grid, st);
  }
}

}  // namespace

extern "C" gfmc_status gfmc_stream_bandwidth(int32_t mode, const void* a, const void* b, void* c,
                                             size_t bytes, int32_t reps, void* stream,
                                             double* gbs) {
  if (mode < 0 || mode > 3) return gfmc_fail(GFMC_EINVAL, "mode must be 0..3");
  if (reps < 1 || !gbs) return gfmc_fail(GFMC_EINVAL, "reps must be >= 1 and gbs non-NULL");
  if (bytes < 16 || (bytes & 15)) return gfmc_fail(GFMC_EINVAL, "bytes must be a multiple of 16");
  if (!c || (mode != 1 && !a) || (mode == 3 && !b))
    return gfmc_fail(GFMC_EINVAL, "buffer missing for this mode");
  const size_t n = bytes / 16;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t want = (n + (size_t)kUnroll * 256 - 1) / ((size_t)kUnroll * 256);
  const f4* fa = (const f4*)a;
  const f4* fb = (const f4*)b;
  f4* fc = (f4*)c;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return gfmc_fail(GFMC_EDEVICE, "hipEventCreate failed");
  }
  const double per = (mode <= 1) ? 1.0 : (mode == 2 ? 2.0 : 3.0);
  double best = 0.0;
  hipError_t e = hipSuccess;
  for (int bpc : {2, 4, 8, 16}) {
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(want, (size_t)cus * bpc));
    e = launch_mode(mode, fa, fb, fc, n, grid, st);   // warm-up pass
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_mode(mode, fa, fb, fc, n, grid, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    best = std::max(best, per * (double)bytes * reps / (ms * 1e-3) / 1e9);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return gfmc_fail(GFMC_EDEVICE, std::string("stream probe: ") + hipGetErrorString(e));
  *gbs = best;
  return GFMC_OK;
}
