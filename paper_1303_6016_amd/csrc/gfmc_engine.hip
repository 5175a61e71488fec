// gfmc_engine.hip -- serving engine of the C ABI (include/gfmc.h, "serving"):
// continuous batching of independent chain requests on one device.
//
// A host worker thread owns the device streams.  Running chains are grouped
// by precision x start-vector form x hopping mode x kernel shape (LDS-resident
// or multi-block); each group has a launch plan, and the groups with members
// are dealt over two streams, created when first needed, so that two run side
// by side.  With its own stream the engine uses at most three, which leaves
// the caller's stream a hardware queue of its own among the four a process
// gets by default.  Each iteration the worker (1) admits queued
// requests in arrival order while a slot and a large enough block of the HBM
// budget are free; a request that does not fit lets later ones that do in
// ahead of it, until it has waited kHoldAfter seconds, after which admission
// holds for it (no request is starved); (2) retires cancelled requests, (3) re-uploads the plans
// when the set of running chains changed, (4) advances every group by a
// number of proposals inversely proportional to the estimated device time of
// one of its proposals (capped, and never past a member's sweep boundary),
// each proposal one batched launch sequence over the group's chains, and
// (5) at each chain's sweep boundary measures |m| and records the sweep's wall
// time.  Per-chain arithmetic does not depend on which chains share a plan.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "gfmc_host.h"

namespace {

// First-fit allocator over the engine's device allocation, 256-byte blocks.
struct Arena {
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  void init(size_t n) {
    size = n;
    used = 0;
    free_.clear();
    free_[0] = n;
  }
  bool fits(size_t n) const {
    n = align256(n);
    for (const auto& kv : free_)
      if (kv.second >= n) return true;
    return false;
  }
  bool alloc(size_t n, size_t& off) {
    n = align256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align256(n);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  uint64_t id = 0;
  gfmc_chain_params p;
  Derived d;
  int init = 0;
  double frac = 0;
  int nsweeps = 1;
  double t_submit = 0, t_admit = -1, t_first_sweep = -1, t_sweep_start = 0;
  bool cancel = false;
  gfmc_chain* chain = nullptr;
  size_t off = 0, bytes = 0;
  int64_t done_props = 0;
  int64_t step_props = 0;   // proposals enqueued for it in the current iteration
  int sweeps = 0;
  double mag_last = 0, mag_sum = 0;
};

}  // namespace

// Chains of one precision x start-vector form x hopping mode x kernel shape
// (LDS-resident or multi-block) share a launch plan; its descriptor table is
// re-uploaded only when its members change.  Keeping the shapes apart lets
// small chains run one launch per proposal while large ones run M/2.
constexpr int kGroups = 16;
constexpr int kStreams = 2;              // group streams (plus the engine's own)
constexpr int kMaxReps = 64;             // proposals per group and iteration
struct Group {
  Plan plan;
  int slot = -1;                      // group stream in use (-1: none yet)
  std::vector<gfmc_chain*> members;   // plan order (most Chebyshev steps first)
  std::vector<Request*> reqs;         // the members' requests
  double cost = 0;                    // estimated device time of one proposal (us)
  int reps = 1;                       // proposals per iteration
};

static int group_of(const Derived& d) {
  return d.fp32 | (d.ov << 1) | (d.hops << 2) | (resident_ok(d) ? 8 : 0);
}

// Estimated device time of one proposal of a group, in microseconds, from
// the measured kernel costs on this chip: a fixed ~40 us for the proposal,
// moment-assembly, reconstruction and spinor launches; the resident kernel
// runs one workgroup per chain side by side, a step taking about
// 0.1 + 0.95 x (items per thread) us (1.0 us at 4^3, 2.2-2.6 us at 8^3,
// 3.9 us at 10^3); the
// multi-block path runs one launch per step over the chains still stepping,
// about 4.4 us + 0.034 ns (FP32) or 0.069 ns (FP64) per site pair, at least
// 6 us.
static double proposal_cost(const Plan& P, const std::vector<gfmc_chain*>& m) {
  constexpr double kFixed = 40.0;
  double c = 0;
  if (P.resident) {
    for (auto* ch : m) {
      const double items = std::ceil(7.0 * ch->d.half / kResThreads);
      c = std::max(c, ch->d.S * (0.1 + 0.95 * items));
    }
    return kFixed + c;
  }
  const double per_pair = P.fp32 ? 3.4e-5 : 6.9e-5;
  const double pairs_per_block = (double)kStepThreads * std::max(P.ppt, 1);
  int nact = P.n;
  for (int s = 1; s <= P.smax; ++s) {
    while (nact > 0 && P.S[nact - 1] < s) --nact;
    c += std::max(6.0, 4.4 + per_pair * pairs_per_block * P.blkoff[nact]);
  }
  return kFixed + c;
}

struct gfmc_engine {
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  char* base = nullptr;
  char* plan_mem = nullptr;
  hipStream_t stream = nullptr;         // admissions, |m|, read-backs
  hipStream_t gstream[kStreams] = {};   // dealt over the groups with members
  Arena arena;
  Group groups[kGroups];
  bool members_changed = true;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::vector<Request*> running;
  std::vector<gfmc_result> done;
  std::vector<std::pair<double, uint64_t>> lat;
  std::thread worker;
  bool stop = false;
  bool busy = false;          // worker is between admission and retirement
  uint64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  gfmc_status fatal = GFMC_OK;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

static size_t plan_bytes(int n) {
  return align256((size_t)n * sizeof(Desc)) + align256((size_t)(n + 1) * sizeof(int)) +
         align256((size_t)n * sizeof(int)) + align256((size_t)(2 * n + 8) * sizeof(int)) +
         align256((size_t)kRecCap * n * sizeof(int32_t)) +
         align256((size_t)kRecCap * n * sizeof(gfmc_step_record)) +
         align256((size_t)kMagCap * n * sizeof(double));
}

static gfmc_result make_result(const Request* r, gfmc_status st, int64_t accepted, double t) {
  gfmc_result x;
  memset(&x, 0, sizeof(x));
  x.request_id = r->id;
  x.status = st;
  x.L = r->p.L;
  x.M = r->p.M;
  x.sweeps = r->sweeps;
  x.proposals = r->done_props;
  x.accepted = accepted;
  x.magnetization = r->mag_last;
  x.magnetization_mean = r->sweeps ? r->mag_sum / r->sweeps : 0.0;
  x.t_submit = r->t_submit;
  x.t_admit = r->t_admit;
  x.t_first_sweep = r->t_first_sweep;
  x.t_done = t;
  return x;
}

// Retire a running request (caller holds no lock; the worker thread only).
// Wait for all device work of the engine (every group stream and the
// engine's own stream).
static hipError_t sync_all(gfmc_engine* E) {
  hipError_t e = hipSuccess;
  for (int g = 0; g < kStreams; ++g)
    if (E->gstream[g]) {
      const hipError_t eg = hipStreamSynchronize(E->gstream[g]);
      if (e == hipSuccess) e = eg;
    }
  const hipError_t e0 = hipStreamSynchronize(E->stream);
  return e == hipSuccess ? e0 : e;
}

static void retire(gfmc_engine* E, Request* r, gfmc_status st) {
  // the chain's last proposals may still be queued: wait before its memory is reused
  if (sync_all(E) != hipSuccess && st == GFMC_OK) st = GFMC_EDEVICE;
  int64_t acc = 0;
  if (r->chain) {
    if (hipMemcpyAsync(&acc, &r->chain->desc.ctl->accepted_total, 8, hipMemcpyDeviceToHost,
                       E->stream) != hipSuccess ||
        hipStreamSynchronize(E->stream) != hipSuccess)
      acc = -1;
  }
  const gfmc_result res = make_result(r, st, acc, E->now());
  std::lock_guard<std::mutex> g(E->mu);
  E->done.push_back(res);
  if (r->chain) {
    delete r->chain;
    r->chain = nullptr;
    E->arena.release(r->off, r->bytes);
  }
  E->running.erase(std::remove(E->running.begin(), E->running.end(), r), E->running.end());
  E->members_changed = true;
  delete r;
}

// Rebuild the member lists of the groups after admissions or retirements and
// re-upload every non-empty plan (a new chain may reuse the host address of a
// retired one, so equal pointer lists do not mean equal descriptors).
static gfmc_status refresh_groups(gfmc_engine* E) {
  for (int g = 0; g < kGroups; ++g) E->groups[g].reqs.clear();
  for (auto* r : E->running) E->groups[group_of(r->d)].reqs.push_back(r);
  // deal the groups with members over the streams in group order; a group
  // that changes stream may still have work queued on its old one that reads
  // its plan tables, so all streams drain first
  int k = 0;
  bool moved = false;
  int slot[kGroups];
  for (int g = 0; g < kGroups; ++g) {
    slot[g] = E->groups[g].reqs.empty() ? -1 : (k++ % kStreams);
    moved |= slot[g] >= 0 && E->groups[g].slot >= 0 && slot[g] != E->groups[g].slot;
  }
  if (moved && sync_all(E) != hipSuccess) return gfmc_fail(GFMC_EDEVICE, "stream sync failed");
  for (int g = 0; g < kGroups; ++g) {
    if (slot[g] < 0) continue;
    if (!E->gstream[slot[g]])
      HIPCHK(hipStreamCreateWithFlags(&E->gstream[slot[g]], hipStreamNonBlocking));
    E->groups[g].slot = slot[g];
    E->groups[g].plan.stream = E->gstream[slot[g]];
  }
  for (int g = 0; g < kGroups; ++g) {
    Group& G = E->groups[g];
    // plan order: most Chebyshev steps first (requests and chains alike)
    std::stable_sort(G.reqs.begin(), G.reqs.end(),
                     [](const Request* a, const Request* b) { return a->d.S > b->d.S; });
    std::vector<gfmc_chain*> L;
    for (auto* r : G.reqs) L.push_back(r->chain);
    G.members = L;
    if (L.empty()) continue;
    plan_shape(G.plan, L);
    CHK(upload_plan(G.plan, L));
    G.cost = proposal_cost(G.plan, L);
  }
  E->members_changed = false;
  return GFMC_OK;
}

// One iteration: every group advances its chains by about reps proposals,
// reps about the ratio of the costliest group's proposal to its own (so
// chains of every size progress at a similar device-time rate), at most
// kMaxReps, and no chain past its next sweep boundary (|m| is taken there).
// LDS-resident groups run reps lock-step proposals.  Multi-block groups run
// a step-granular window of reps x (their most steps) rounds: the chains with
// the most steps make reps proposals and every other chain as many as fit,
// each restarting as soon as its last proposal is reconstructed, capped at
// its sweep boundary.
static gfmc_status iterate(gfmc_engine* E) {
  if (E->members_changed) CHK(refresh_groups(E));
  double cmax = 0;
  for (int g = 0; g < kGroups; ++g)
    if (!E->groups[g].members.empty()) cmax = std::max(cmax, E->groups[g].cost);
  for (int g = 0; g < kGroups; ++g) {
    Group& G = E->groups[g];
    if (G.members.empty()) continue;
    int reps = (int)std::min((double)kMaxReps, std::max(1.0, cmax / std::max(G.cost, 1.0)));
    if (G.plan.cont && !G.plan.resident) {
      // members are in plan order (most steps first), as the plan's tables
      const int n = (int)G.members.size();
      std::vector<int> cap(n), props(n);
      int64_t rmax = 0;
      for (int i = 0; i < n; ++i) {
        const Request* r = G.reqs[i];
        cap[i] = (int)std::min<int64_t>(kMaxReps * 64, r->d.N - r->done_props % r->d.N);
        rmax = std::max<int64_t>(rmax, (int64_t)cap[i] * r->d.S);
      }
      // the window never outlasts every chain's sweep boundary
      const int rounds = (int)std::min<int64_t>((int64_t)reps * G.plan.smax, rmax);
      CHK(enqueue_window(G.plan, rounds, cap.data(), props.data()));
      for (int i = 0; i < n; ++i) G.reqs[i]->step_props = props[i];
      G.reps = reps;
    } else {
      for (auto* r : G.reqs)
        reps = (int)std::min<int64_t>(reps, r->d.N - r->done_props % r->d.N);
      G.reps = reps;
      for (int k = 0; k < reps; ++k) CHK(enqueue_proposal(G.plan, nullptr, nullptr, true));
      for (auto* r : G.reqs) r->step_props = reps;
    }
  }
  return GFMC_OK;
}

// A queued request that has waited kHoldAfter seconds without fitting the
// free budget holds admission: the requests behind it wait until it is in.
constexpr double kHoldAfter = 10.0;
static bool held(const gfmc_engine* E, const Request* r) {
  return E->now() - r->t_submit >= kHoldAfter;
}

// Whether the admission pass would take a queued request now (caller holds
// the engine's lock): a free slot and a request that fits, scanning in
// arrival order up to the first held one.
static bool admissible(const gfmc_engine* E) {
  if ((int)E->running.size() >= E->max_slots) return false;
  for (const Request* r : E->queue) {
    if (E->arena.fits(r->bytes)) return true;
    if (held(E, r)) return false;
  }
  return false;
}

static void worker_main(gfmc_engine* E) {
  (void)hipSetDevice(E->device);
  std::vector<Request*> admitted;
  int since_sync = 0;
  while (true) {
    admitted.clear();
    {
      std::unique_lock<std::mutex> lk(E->mu);
      if (E->stop) break;
      for (auto it = E->queue.begin();
           it != E->queue.end() && (int)(E->running.size() + admitted.size()) < E->max_slots;) {
        Request* r = *it;
        size_t off = 0;
        if (E->arena.alloc(r->bytes, off)) {
          r->off = off;
          it = E->queue.erase(it);
          admitted.push_back(r);
        } else if (held(E, r)) {
          break;   // later requests wait until this one is admitted
        } else {
          ++it;    // later, smaller requests may go first
        }
      }
      if (E->running.empty() && admitted.empty()) {
        E->busy = false;
        E->cv.notify_all();
        E->cv.wait(lk, [&] { return E->stop || !E->queue.empty(); });
        continue;
      }
      E->busy = true;
    }
    for (auto* r : admitted) {
      gfmc_chain* c = new (std::nothrow) gfmc_chain();
      gfmc_status st = c ? chain_setup(c, &r->p, r->d, E->base + r->off, r->bytes, E->stream)
                         : GFMC_ENOMEM;
      if (st == GFMC_OK) st = chain_init_spins(c, r->init, r->frac);
      if (st == GFMC_OK && hipStreamSynchronize(E->stream) != hipSuccess) st = GFMC_EDEVICE;
      std::lock_guard<std::mutex> g(E->mu);
      if (st != GFMC_OK) {
        delete c;
        E->arena.release(r->off, r->bytes);
        E->done.push_back(make_result(r, st, 0, E->now()));
        delete r;
        continue;
      }
      r->chain = c;
      r->t_admit = E->now();
      r->t_sweep_start = r->t_admit;
      E->running.push_back(r);
      E->members_changed = true;
    }
    // cancelled requests leave before the next proposal
    std::vector<Request*> cancelled;
    {
      std::lock_guard<std::mutex> g(E->mu);
      for (auto* r : E->running)
        if (r->cancel) cancelled.push_back(r);
    }
    for (auto* r : cancelled) retire(E, r, GFMC_ECANCELED);
    if (E->running.empty()) continue;

    gfmc_status st = iterate(E);
    // The host knows every chain's proposal count, so it waits for the device
    // only where it needs device results or time stamps: sweep boundaries,
    // pending admissions or cancellations, and every 8th iteration (so that
    // queued requests are not kept behind a long run of enqueued work).
    bool boundary_now = false, pending = false;
    for (auto* r : E->running)
      boundary_now |= r->step_props > 0 && ((r->done_props + r->step_props) % r->d.N == 0);
    {
      std::lock_guard<std::mutex> g(E->mu);
      pending = admissible(E);
      for (auto* r : E->running) pending |= r->cancel;
    }
    ++since_sync;
    if (st == GFMC_OK && (boundary_now || pending || since_sync >= 8)) {
      if (sync_all(E) != hipSuccess) st = GFMC_EDEVICE;
      since_sync = 0;
    }
    if (st != GFMC_OK) {
      std::vector<Request*> all = E->running;
      for (auto* r : all) retire(E, r, st);
      std::lock_guard<std::mutex> g(E->mu);
      E->fatal = st;
      E->stop = true;
      break;
    }
    const double t = E->now();
    std::vector<Request*> boundary;
    for (auto* r : E->running) {
      const int64_t k = r->step_props;
      r->done_props += k;
      r->step_props = 0;
      if (k > 0 && r->done_props % r->d.N == 0) boundary.push_back(r);
    }
    if (boundary.empty()) continue;
    std::vector<double> mags(boundary.size());
    bool ok = true;
    for (size_t i = 0; i < boundary.size(); ++i) {
      Plan& cp = boundary[i]->chain->plan;
      ok = ok && launch_magnetization(cp.d_desc, 1, cp.d_mag, E->stream) == hipSuccess &&
           hipMemcpyAsync(&mags[i], cp.d_mag, 8, hipMemcpyDeviceToHost, E->stream) == hipSuccess;
    }
    ok = ok && hipStreamSynchronize(E->stream) == hipSuccess;
    std::vector<Request*> finished;
    {
      std::lock_guard<std::mutex> g(E->mu);
      for (size_t i = 0; i < boundary.size(); ++i) {
        Request* r = boundary[i];
        E->lat.push_back({t - r->t_sweep_start, r->id});
        r->t_sweep_start = t;
        r->sweeps += 1;
        r->mag_last = mags[i];
        r->mag_sum += mags[i];
        if (r->t_first_sweep < 0) r->t_first_sweep = t;
        if (r->sweeps >= r->nsweeps) finished.push_back(r);
      }
    }
    for (auto* r : finished) retire(E, r, ok ? GFMC_OK : GFMC_EDEVICE);
  }
  // stop: cancel whatever is still running
  std::vector<Request*> all = E->running;
  for (auto* r : all) retire(E, r, GFMC_ECANCELED);
  std::lock_guard<std::mutex> g(E->mu);
  E->busy = false;
  E->cv.notify_all();
}

extern "C" {

gfmc_status gfmc_engine_create(int device, size_t budget, int32_t max_slots, gfmc_engine** out) {
  if (!out) return gfmc_fail(GFMC_EINVAL, "out is NULL");
  if (max_slots < 1 || max_slots > 4096) return gfmc_fail(GFMC_EINVAL, "max_slots in [1, 4096]");
  if (budget < 4096) return gfmc_fail(GFMC_EINVAL, "hbm_budget_bytes too small");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return gfmc_fail(GFMC_EINVAL, "no such device");
  HIPCHK(hipSetDevice(device));
  gfmc_engine* E = new (std::nothrow) gfmc_engine();
  if (!E) return gfmc_fail(GFMC_ENOMEM, "host allocation failed");
  E->device = device;
  E->budget = budget & ~(size_t)255;
  E->max_slots = max_slots;
  E->t0 = std::chrono::steady_clock::now();
  if (hipMalloc(&E->base, E->budget) != hipSuccess) {
    delete E;
    return gfmc_fail(GFMC_ENOMEM, "hipMalloc of the HBM budget failed");
  }
  bool ok = hipMalloc(&E->plan_mem, kGroups * plan_bytes(max_slots)) == hipSuccess &&
            hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    if (E->stream) (void)hipStreamDestroy(E->stream);
    (void)hipFree(E->base);
    if (E->plan_mem) (void)hipFree(E->plan_mem);
    delete E;
    return gfmc_fail(GFMC_EDEVICE, "engine device setup failed");
  }
  E->arena.init(E->budget);
  const size_t pb = plan_bytes(max_slots);
  for (int g = 0; g < kGroups; ++g) {
    Plan& P = E->groups[g].plan;
    char* w = E->plan_mem + g * pb;
    P.stream = nullptr;   // a group stream is dealt when the group gains members
    P.fp32 = g & 1;
    P.ov = (g >> 1) & 1;
    P.hops = (g >> 2) & 1;
    P.ppt = (g & 8) ? 0 : 1;   // LDS-resident groups, else one site pair per thread
    P.d_desc = (Desc*)w; w += align256((size_t)max_slots * sizeof(Desc));
    P.d_blkoff = (int*)w; w += align256((size_t)(max_slots + 1) * sizeof(int));
    P.d_act_end = (int*)w; w += align256((size_t)max_slots * sizeof(int));
    P.d_coh_blkoff = (int*)w; w += align256((size_t)(2 * max_slots + 8) * sizeof(int));
    P.cont = (g & 8) ? 0 : 1;   // multi-block groups: step-granular windows
    P.d_force = (int32_t*)w; w += align256((size_t)kRecCap * max_slots * sizeof(int32_t));
    P.d_rec = (gfmc_step_record*)w;
    w += align256((size_t)kRecCap * max_slots * sizeof(gfmc_step_record));
    P.d_mag = (double*)w;
  }
  E->worker = std::thread(worker_main, E);
  *out = E;
  return GFMC_OK;
}

gfmc_status gfmc_engine_submit(gfmc_engine* E, const gfmc_chain_params* p, gfmc_init init,
                               double frac, int32_t nsweeps, uint64_t* id) {
  if (!E || !id) return gfmc_fail(GFMC_EINVAL, "NULL argument");
  Derived d;
  CHK(derive(p, d));
  if (nsweeps < 1) return gfmc_fail(GFMC_EINVAL, "nsweeps must be >= 1");
  const int32_t im = gfmc_enum_value(init);
  if (im != GFMC_INIT_RANDOM && im != GFMC_INIT_FM && im != GFMC_INIT_FM_PLUS_RANDOM)
    return gfmc_fail(GFMC_EINVAL, "unknown init mode");
  if (init == GFMC_INIT_FM_PLUS_RANDOM && !(frac >= 0 && frac <= 1))
    return gfmc_fail(GFMC_EINVAL, "random_fraction must be in [0, 1]");
  const size_t need = layout_of(d).total;
  if (align256(need) > E->budget) return gfmc_fail(GFMC_EBUSY, "request exceeds the HBM budget");
  Request* r = new (std::nothrow) Request();
  if (!r) return gfmc_fail(GFMC_ENOMEM, "host allocation failed");
  r->p = *p;
  r->d = d;
  r->init = init;
  r->frac = frac;
  r->nsweeps = nsweeps;
  r->bytes = need;
  std::lock_guard<std::mutex> g(E->mu);
  if (E->stop) {
    delete r;
    return gfmc_fail(E->fatal != GFMC_OK ? E->fatal : GFMC_ESTATE, "engine stopped");
  }
  r->id = E->next_id++;
  r->t_submit = E->now();
  E->queue.push_back(r);
  *id = r->id;
  E->cv.notify_all();
  return GFMC_OK;
}

gfmc_status gfmc_engine_poll(gfmc_engine* E, gfmc_result* out, int32_t cap, int32_t* n) {
  if (!E || !n || cap < 0 || (cap > 0 && !out)) return gfmc_fail(GFMC_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> g(E->mu);
  const int k = std::min<int>(cap, (int)E->done.size());
  for (int i = 0; i < k; ++i) out[i] = E->done[i];
  E->done.erase(E->done.begin(), E->done.begin() + k);
  *n = k;
  return GFMC_OK;
}

gfmc_status gfmc_engine_cancel(gfmc_engine* E, uint64_t id) {
  if (!E) return gfmc_fail(GFMC_EINVAL, "engine is NULL");
  std::lock_guard<std::mutex> g(E->mu);
  for (auto it = E->queue.begin(); it != E->queue.end(); ++it) {
    if ((*it)->id == id) {
      Request* r = *it;
      E->queue.erase(it);
      E->done.push_back(make_result(r, GFMC_ECANCELED, 0, E->now()));
      delete r;
      E->cv.notify_all();
      return GFMC_OK;
    }
  }
  for (auto* r : E->running)
    if (r->id == id) {
      r->cancel = true;
      return GFMC_OK;
    }
  return gfmc_fail(GFMC_EINVAL, "unknown or finished request id");
}

gfmc_status gfmc_engine_sweep_latencies(gfmc_engine* E, double* sec, uint64_t* ids, int32_t cap,
                                        int32_t* n) {
  if (!E || !n || cap < 0 || (cap > 0 && !sec)) return gfmc_fail(GFMC_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> g(E->mu);
  const int k = std::min<int>(cap, (int)E->lat.size());
  for (int i = 0; i < k; ++i) {
    sec[i] = E->lat[i].first;
    if (ids) ids[i] = E->lat[i].second;
  }
  E->lat.erase(E->lat.begin(), E->lat.begin() + k);
  *n = k;
  return GFMC_OK;
}

gfmc_status gfmc_engine_status(gfmc_engine* E, int32_t* queued, int32_t* running,
                               int32_t* finished, size_t* bytes_in_use) {
  if (!E) return gfmc_fail(GFMC_EINVAL, "engine is NULL");
  std::lock_guard<std::mutex> g(E->mu);
  if (queued) *queued = (int32_t)E->queue.size();
  if (running) *running = (int32_t)E->running.size();
  if (finished) *finished = (int32_t)E->done.size();
  if (bytes_in_use) *bytes_in_use = E->arena.used;
  return GFMC_OK;
}

gfmc_status gfmc_engine_drain(gfmc_engine* E, double timeout_s) {
  if (!E) return gfmc_fail(GFMC_EINVAL, "engine is NULL");
  std::unique_lock<std::mutex> lk(E->mu);
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                         std::chrono::duration<double>(timeout_s));
  const bool ok = E->cv.wait_until(lk, until, [&] {
    return E->stop || (E->queue.empty() && E->running.empty() && !E->busy);
  });
  if (E->fatal != GFMC_OK) return gfmc_fail(E->fatal, "engine stopped after a device error");
  return ok ? GFMC_OK : gfmc_fail(GFMC_EBUSY, "drain timed out");
}

gfmc_status gfmc_engine_destroy(gfmc_engine* E) {
  if (!E) return GFMC_OK;
  {
    std::lock_guard<std::mutex> g(E->mu);
    E->stop = true;
    for (auto* r : E->queue) delete r;
    E->queue.clear();
    E->cv.notify_all();
  }
  if (E->worker.joinable()) E->worker.join();
  (void)hipSetDevice(E->device);
  (void)sync_all(E);
  for (int g = 0; g < kStreams; ++g)
    if (E->gstream[g]) (void)hipStreamDestroy(E->gstream[g]);
  (void)hipStreamDestroy(E->stream);
  (void)hipFree(E->plan_mem);
  (void)hipFree(E->base);
  delete E;
  return GFMC_OK;
}

}  // extern "C"
