// capi_sanitize_driver.cpp -- TEST INFRASTRUCTURE ONLY.  Calls the host side
// of the C ABI (include/gfmc.h) on a machine with no visible GPU, so that a
// build of the library's host code with AddressSanitizer, LeakSanitizer and
// UndefinedBehaviorSanitizer (tests/test_capi_sanitizers.py) checks its
// parameter validation, workspace sizing and error paths for memory errors,
// leaks and undefined behaviour:
//   * status strings, version, last-error text;
//   * gfmc_workspace_bytes over a grid of valid and invalid parameters
//     (both precisions, every start-vector form and hopping mode, both
//     kernels, odd and out-of-range L, M and K, bad beta, t and b), printing a checksum of the sizes;
//   * NULL handles and bad arguments on every entry point that takes them;
//   * chain, engine and allocation-free ΔS_eff calls that pass validation
//     and then fail at their first device call (no device), which must
//     release what they allocated on the host.
// Prints one line per section and exits 0 when every status is as expected.
// Refuses to run where a device is visible: the error-path section passes a
// workspace address that is not device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>

#include "gfmc.h"

static int bad = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s (last error: %s)\n", what, gfmc_last_error());
    bad = 1;
  }
}

static gfmc_chain_params base(int L, int M, int prec) {
  gfmc_chain_params p;
  std::memset(&p, 0, sizeof p);
  p.L = L;
  p.t = 1.0;
  p.beta = 20.0;
  p.mu = 0.0;
  p.M = M;
  p.K = 0;
  p.kernel = GFMC_JACKSON;
  p.lorentz_lambda = 4.0;
  p.scale_a = 0.0;
  p.scale_b = 0.0;
  p.precision = (gfmc_precision)prec;
  p.proposal = GFMC_PROPOSE_SPHERE;
  p.cone_angle = 0.3;
  p.seed = 3;
  p.chain_id = 1;
  return p;
}

int main() {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    std::printf("a device is visible: this driver runs only without one\n");
    return 3;
  }

  // status strings
  for (int32_t s = -9; s <= 9; ++s) expect(gfmc_status_string(s) != nullptr, "status string");
  expect(gfmc_version() && std::strlen(gfmc_version()) > 0, "version");
  std::printf("strings ok\n");

  // workspace sizes over valid and invalid parameters
  uint64_t sum = 0;
  int nvalid = 0, ninvalid = 0;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int L : {1, 2, 3, 4, 6, 8, 10, 16, 32, 64, 255, 256, 258}) {
    for (int M : {0, 2, 3, 64, 256, 2048, 8192, 8194}) {
      for (int prec : {0, 1}) {
        for (int vec : {0, 1, 2}) {
          for (int hops : {0, 1}) {
            gfmc_chain_params p = base(L, M, prec);
            p.vectors = (gfmc_vectors)vec;
            p.hoppings = (gfmc_hoppings)hops;
            p.kernel = (L + M) & 1 ? GFMC_LORENTZ : GFMC_JACKSON;
            p.K = (M % 3 == 0) ? 3 * M : 2 * M;   // some K not a power of two
            size_t bytes = 0;
            const gfmc_status st = gfmc_workspace_bytes(&p, &bytes);
            if (st == GFMC_OK) {
              expect(bytes > 0 && bytes % 256 == 0, "workspace bytes aligned");
              sum = sum * 1000003u + bytes;
              ++nvalid;
            } else {
              expect(st == GFMC_EINVAL && gfmc_last_error()[0] != 0, "invalid parameters -> EINVAL");
              ++ninvalid;
            }
          }
        }
      }
    }
  }
  for (double beta : {0.0, -1.0, nan, 1e300}) {
    gfmc_chain_params p = base(8, 64, 0);
    p.beta = beta;
    size_t bytes = 0;
    const gfmc_status st = gfmc_workspace_bytes(&p, &bytes);
    if (st == GFMC_OK) sum = sum * 1000003u + bytes; else ++ninvalid;
  }
  // enum fields holding values outside their enums (as a C caller may pass)
  const int32_t bad_enum[5][2] = {{0, 2}, {1, 5}, {2, -1}, {3, 7}, {4, 3}};
  for (const auto& be : bad_enum) {
    gfmc_chain_params p = base(8, 64, 0);
    void* field[5] = {&p.precision, &p.kernel, &p.proposal, &p.vectors, &p.hoppings};
    std::memcpy(field[be[0]], &be[1], sizeof(int32_t));
    size_t bytes = 0;
    expect(gfmc_workspace_bytes(&p, &bytes) == GFMC_EINVAL, "enum field out of range -> EINVAL");
    ++ninvalid;
  }
  gfmc_chain_params pb = base(8, 64, 0);
  pb.t = nan;
  size_t dummy = 0;
  expect(gfmc_workspace_bytes(&pb, &dummy) == GFMC_EINVAL, "NaN t");
  pb = base(8, 64, 0);
  pb.scale_b = 0.5;
  expect(gfmc_workspace_bytes(&pb, &dummy) == GFMC_EINVAL, "b != 0");
  expect(gfmc_workspace_bytes(nullptr, &dummy) == GFMC_EINVAL, "NULL params");
  pb = base(8, 64, 0);
  expect(gfmc_workspace_bytes(&pb, nullptr) == GFMC_EINVAL, "NULL bytes");
  std::printf("workspace sizes: %d valid, %d invalid, checksum %llu\n", nvalid, ninvalid,
              (unsigned long long)sum);

  // NULL handles and bad arguments
  int32_t i32 = 0;
  int64_t i64 = 0;
  double d = 0.0, buf[8] = {0};
  size_t sz = 0;
  expect(gfmc_chain_destroy(nullptr) == GFMC_OK, "destroy NULL chain");
  expect(gfmc_batch_destroy(nullptr) == GFMC_OK, "destroy NULL batch");
  expect(gfmc_set_params(nullptr, 1.0, 1.0, 0.0) == GFMC_EINVAL, "set_params NULL");
  expect(gfmc_init_spins(nullptr, GFMC_INIT_RANDOM, 0.0) == GFMC_EINVAL, "init_spins NULL");
  expect(gfmc_set_spins(nullptr, buf, buf) == GFMC_EINVAL, "set_spins NULL");
  expect(gfmc_get_spins(nullptr, buf, buf) == GFMC_EINVAL, "get_spins NULL");
  expect(gfmc_set_counter(nullptr, 0) == GFMC_EINVAL, "set_counter NULL");
  expect(gfmc_get_counter(nullptr, &i64) == GFMC_EINVAL, "get_counter NULL");
  expect(gfmc_chain_nonfinite(nullptr, &i64) == GFMC_EINVAL, "nonfinite NULL");
  expect(gfmc_moments(nullptr, 0, buf) == GFMC_EINVAL, "moments NULL");
  expect(gfmc_pair_moments(nullptr, 0, 1.0, 1.0, buf) == GFMC_EINVAL, "pair_moments NULL");
  expect(gfmc_mixed_moments(nullptr, 0, 1.0, 1.0, buf) == GFMC_EINVAL, "mixed_moments NULL");
  expect(gfmc_delta_seff(nullptr, 0, 1.0, 1.0, &d, &d) == GFMC_EINVAL, "delta_seff NULL");
  expect(gfmc_step(nullptr, -1, nullptr) == GFMC_EINVAL, "step NULL");
  expect(gfmc_sweep(nullptr, 1, buf, &i64) == GFMC_EINVAL, "sweep NULL");
  expect(gfmc_magnetization(nullptr, &d) == GFMC_EINVAL, "magnetization NULL");
  expect(gfmc_sync(nullptr) == GFMC_EINVAL, "sync NULL");
  expect(gfmc_chain_step_bytes(nullptr, &d, &i32) == GFMC_EINVAL, "step_bytes NULL");
  expect(gfmc_batch_workspace_bytes(nullptr, 0, &sz) == GFMC_EINVAL, "batch bytes NULL");
  gfmc_batch* bh = nullptr;
  expect(gfmc_batch_create(nullptr, 0, nullptr, 0, nullptr, &bh) == GFMC_EINVAL, "batch NULL");
  expect(gfmc_batch_step(nullptr, 1, nullptr, nullptr) == GFMC_EINVAL, "batch step NULL");
  expect(gfmc_batch_set_tuning(nullptr, 1) == GFMC_EINVAL, "set_tuning NULL");
  expect(gfmc_batch_set_lanes(nullptr, 2) == GFMC_EINVAL, "set_lanes NULL");
  expect(gfmc_batch_set_block_threads(nullptr, 256) == GFMC_EINVAL, "block_threads NULL");
  expect(gfmc_batch_get_tuning(nullptr, &i32, &i32) == GFMC_EINVAL, "get_tuning NULL");
  expect(gfmc_batch_autotune(nullptr, 4, &i32) == GFMC_EINVAL, "autotune NULL");
  expect(gfmc_engine_submit(nullptr, nullptr, GFMC_INIT_RANDOM, 0.0, 1, nullptr) == GFMC_EINVAL,
         "engine submit NULL");
  expect(gfmc_engine_poll(nullptr, nullptr, 0, &i32) == GFMC_EINVAL, "engine poll NULL");
  expect(gfmc_engine_destroy(nullptr) == GFMC_OK, "engine destroy NULL");
  expect(gfmc_stream_bandwidth(7, buf, buf, buf, 64, 1, nullptr, &d) == GFMC_EINVAL, "probe mode");
  expect(gfmc_stream_bandwidth(0, buf, buf, buf, 17, 1, nullptr, &d) == GFMC_EINVAL, "probe size");
  std::printf("null handles ok\n");

  // calls that pass validation and fail at their first device call
  int fails = 0;
  for (int L : {4, 12, 32}) {
    for (int prec : {0, 1}) {
      gfmc_chain_params p = base(L, 64, prec);
      size_t bytes = 0;
      expect(gfmc_workspace_bytes(&p, &bytes) == GFMC_OK, "workspace bytes");
      gfmc_chain* c = nullptr;
      const gfmc_status st =
          gfmc_chain_create(&p, reinterpret_cast<void*>(uintptr_t(1) << 40), bytes, nullptr, &c);
      expect(st != GFMC_OK && c == nullptr, "chain create without a device fails cleanly");
      fails += st != GFMC_OK;
    }
  }
  {
    gfmc_chain_params p = base(8, 64, 0);
    double* fake = reinterpret_cast<double*>(uintptr_t(1) << 40);
    expect(gfmc_delta_seff_static(&p, fake, fake, 3, 1.0, 2.0, fake, fake, nullptr) != GFMC_OK,
           "static delta_seff without a device fails cleanly");
  }
  gfmc_engine* e = nullptr;
  expect(gfmc_engine_create(0, size_t(1) << 30, 8, &e) != GFMC_OK && e == nullptr,
         "engine create without a device fails cleanly");
  std::printf("device error paths: %d chain creations refused\n", fails);

  std::printf(bad ? "driver: FAILED\n" : "driver: clean\n");
  return bad;
}
