"""Benchmark of the GFMC hot path on one MI355X.

Workload (one "step"): one Metropolis proposal on each of 64 independent
chains of a 32^3 periodic cubic lattice, M = 2048 Chebyshev moments, FP32
recursion with FP64 moment sums, temperatures linearly spaced in
[0.02t, 0.2t], uniform-sphere starts from seed 7 (chain_id = chain index).
A proposal runs the whole path: Philox draw, bond changes, M/2 fused
Chebyshev steps over the 7 start vectors, moment assembly, reconstruction
(FFT transform, determinant, phase, energy integral), Metropolis update.

Prints ONE JSON line (rank 0).  value = Chebyshev site-vector updates per
second over the whole job (N * 7 * M/2 per proposal).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

L, M, NCHAIN = 32, 2048, 64
T_LO, T_HI = 0.02, 0.2
SEED = 7
HBM_PEAK_GBS = 8000.0

# Bytes per step round (one Chebyshev step of every chain of the batch; the
# lanes split the same blocks, so the bytes per round do not depend on them)
# that the L2 exchanges with the memory fabric, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (one counter per run), each scaled by what the same counter reads
# for a plain 1 GiB device copy (FETCH x 2.0, WRITE x 1.0); keyed by kernel,
# chains of 32^3, site pairs per thread, non-temporal access and threads per
# block, and valid only for the kernel source they were taken with (sha256
# below), else null.
TRAFFIC_KERNEL_SHA256 = "cd724c4b8cd1d91da370ddf8b45a547aa759edef0ade26e74016a2ccc4ac84a6"
TRAFFIC_BYTES = {("k_step<float>", 64, 2, 0, 256): 213828771,
                 ("k_step_ov<float>", 64, 2, 0, 256): 84205354,
                 ("k_step<float>", 64, 1, 0, 256): 211566567,
                 ("k_step<float>", 64, 1, 0, 512): 210792422,
                 ("k_step<float>", 64, 1, 1, 256): 211564647,
                 ("k_step<float>", 64, 1, 1, 512): 210761703,
                 ("k_step<float>", 64, 2, 1, 256): 211637203,
                 ("k_step<float>", 128, 1, 1, 256): 422920466,
                 ("k_step<float>", 128, 1, 1, 512): 421313234,
                 ("k_step<float>", 128, 2, 1, 256): 422548855,
                 ("k_step<double>", 64, 1, 1, 256): 421342034,
                 ("k_step<double>", 64, 1, 1, 512): 420489682,
                 ("k_step<double>", 64, 2, 1, 256): 423743754}


def note(msg: str):
    """Progress line on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-single", action="store_true")
    ap.add_argument("--graph", type=int, default=0, help="replay one proposal as a HIP graph")
    ap.add_argument("--tuning", type=str, default="",
                    help="PPT,LANES[,NT[,BLOCK_THREADS]]: fix the launch shape, step lanes, "
                         "non-temporal access and step-kernel block size instead of autotuning")
    ap.add_argument("--pair", type=int, default=1,
                    help="also time the {o, v} start-vector form on the same workload")
    ap.add_argument("--pair-tuning", type=str, default="",
                    help="PPT,LANES for the pair-form leg (shape 3: two steps per launch); "
                         "default: autotune")
    ap.add_argument("--stored-hops", type=int, default=1,
                    help="also time the stored-hopping A/B variant of the step kernel")
    ap.add_argument("--small", type=int, default=1,
                    help="also time the 4^3 and 16^3 FP64 workloads")
    ap.add_argument("--hbm", type=int, default=1,
                    help="also time the step kernel with working sets above the last-level cache")
    ap.add_argument("--mixed", type=int, default=1,
                    help="also time one 64^3 chain with eight 32^3 chains in one batch")
    ap.add_argument("--chain-sweep", action="store_true",
                    help="step-kernel bandwidth for 8..128 chains of 32^3 (cache residency)")
    ap.add_argument("--serving", type=float, default=0.0,
                    help="run the serving engine for this many seconds of Poisson arrivals")
    ap.add_argument("--serving-leg", type=int, default=1,
                    help="also run 30 s of the small serving mix and report its sweep latencies")
    ap.add_argument("--serving-mix", type=str, default="small", choices=sorted(SERVING_MIXES),
                    help="lattice-size mix of the serving run")
    ap.add_argument("--serving-load", type=float, default=1.0,
                    help="offered load as a fraction of --serving-capacity (mixes without a rate)")
    ap.add_argument("--serving-capacity", type=float, default=0.0,
                    help="capacity in svu/s that sets the arrival rate (mixes without a rate)")
    ap.add_argument("--serving-drain", type=float, default=1e9,
                    help="seconds of drain after the arrivals before the rest is cancelled")
    ap.add_argument("--physics", action="store_true",
                    help="magnetization against temperature on 4^3, 6^3 and 8^3 (M = 256, mu = 0)")
    ap.add_argument("--fp32-accuracy", action="store_true",
                    help="FP32-recursion error against the FP64 path for L = 4..32, M = 512..8192")
    ap.add_argument("--copy-sweep", action="store_true",
                    help="device-copy bandwidth for working sets of 16 MiB .. 2 GiB")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def tune(batch, fixed: str):
    """Autotune the batch, or fix it from "PPT,LANES[,NT[,BLOCK_THREADS]]"."""
    if fixed:
        vals = [int(v) for v in fixed.split(",")]
        ppt, lanes = vals[0], vals[1]
        batch.set_lanes(lanes)
        if len(vals) > 3:
            batch.set_block_threads(vals[3])
        batch.set_tuning(ppt)
        if len(vals) > 2:
            batch.set_nontemporal(bool(vals[2]))
    else:
        batch.autotune(256)   # 256 steps per trial: shapes within a few per cent apart


def traffic_bytes(kernel: str, chains: int, ppt: int, nt: int = 0, bt: int = 256):
    import hashlib
    src = os.path.join(ROOT, "paper_1303_6016_amd", "csrc", "gfmc_kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != TRAFFIC_KERNEL_SHA256:
        return None
    return TRAFFIC_BYTES.get((kernel, chains, ppt, int(nt), int(bt)))


def host_cpu():
    """Model name and core counts of the host the oracle runs on."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model_name": name, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(max_threads: int = 16):
    """The FP64 oracle on a bounded sample of the same workload (32^3,
    M = 2048, uniform-sphere starts, seed 7): one proposal on one thread,
    then one independent chain per host core (at most max_threads), one
    proposal each, run concurrently -- the chain-per-core decomposition;
    plus a few single-thread proposals of the 4^3 and 16^3 workloads.
    The oracle is C called through ctypes, which releases the GIL, so the
    threads run in parallel."""
    import threading
    import oracle
    svu = L ** 3 * 7 * (M // 2)

    def setup(c):
        m = oracle.Model(L=L, M=M, beta=1.0 / T_LO, seed=SEED, chain_id=c)
        th, ph = oracle.init_spins(m, 0)
        return m, th, ph

    m, th, ph = setup(0)
    t0 = time.perf_counter()
    oracle.step(m, th, ph, 0)
    dt1 = time.perf_counter() - t0

    nthr = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    states = [setup(c) for c in range(nthr)]
    gate = threading.Barrier(nthr + 1)

    def work(st):
        gate.wait()
        oracle.step(st[0], st[1], st[2], 0)

    threads = [threading.Thread(target=work, args=(st,)) for st in states]
    for t in threads:
        t.start()
    gate.wait()
    t0 = time.perf_counter()
    for t in threads:
        t.join()
    dtn = time.perf_counter() - t0
    # the small workloads, single thread, a few proposals each
    per = {}
    for key, kw, mode, frac, nprop in (
            ("4cubed_M256", dict(L=4, M=256, beta=20.0, seed=1, chain_id=0), 0, 0.0, 32),
            ("16cubed_M1024_cone", dict(L=16, M=1024, beta=20.0, seed=42, chain_id=0, proposal=1,
                                        cone=0.3), 2, 0.1, 3)):
        mk = oracle.Model(**kw)
        tk, pk = oracle.init_spins(mk, mode, frac)
        t0 = time.perf_counter()
        for idx in range(nprop):
            oracle.step(mk, tk, pk, idx)
        dk = (time.perf_counter() - t0) / nprop
        sv = mk.N * 7 * (mk.M // 2)
        per[key] = {"proposals_per_s": 1.0 / dk, "svu_per_s": sv / dk, "cores": 1,
                    "sample": f"{nprop} proposals"}
    return {"value": nthr * svu / dtn, "unit": "svu/s", "cores": nthr, "kind": "oracle",
            "sample": f"{nthr} independent 32^3 M=2048 chains, one FP64 proposal each on its "
                      f"own host thread, {dtn:.1f} s wall; svu counted as N*7*M/2 per proposal",
            "svu_accounting": "the oracle evaluates every moment from its definition: M-1 "
                              "recursion steps per start vector, no doubling (a CPU code with "
                              "doubling would need M/2); svu/s counts the method's N*7*M/2 per "
                              "proposal, so the oracle's own site-vector rate is ~2x this value",
            "mc_spin_updates_per_s": nthr / dtn,
            "single_core": {"value": svu / dt1, "unit": "svu/s", "cores": 1,
                            "mc_spin_updates_per_s": 1.0 / dt1,
                            "sample": f"1 proposal of one 32^3 M=2048 chain, {dt1:.1f} s"},
            "small_workloads_1_thread": per,
            "host": host_cpu()}


def chain_state_bytes(ch):
    """Bytes a step reads or writes of one chain: the vectors and the spinor
    cache (the per-step working set; the moment partials are written once)."""
    bps, _ = ch.step_bytes()
    prec = 4 if ch.p.precision == 1 else 8
    nvec = 2 if ch.p.vectors else 7
    return ch.p.L ** 3 * (nvec * 2 * prec + 4 * prec)


def hbm_regime(g, torch, dev, fixed: str, nprop: int = 2):
    """The step kernel with working sets well above the 256 MB last-level
    cache: 128 chains of 32^3 in FP32 (302 MB of vectors and spinors) and 64
    chains of 32^3 in FP64 (302 MB), M = 2048, same temperatures and starts
    as the headline; autotuned shape and lanes; the step rounds of `nprop`
    proposals after one warm-up proposal."""
    out = []
    for nch, prec in ((128, g.FP32_ACC64), (64, g.FP64)):
        temps = [T_LO + (T_HI - T_LO) * c / (nch - 1) for c in range(nch)]
        chs = [g.Chain(g.Params(L=L, M=M, beta=1.0 / temps[c], precision=prec, seed=SEED,
                                chain_id=c), device=dev) for c in range(nch)]
        for ch in chs:
            ch.init_spins(g.INIT_RANDOM)
        b = g.Batch(chs)
        tune(b, fixed)
        ppt, lanes = b.tuning()
        nt = b.form()["nontemporal"]
        bt = b.block_threads()
        b.step(1)
        torch.cuda.synchronize()
        ms_tot, nl_tot = 0.0, 0
        for _ in range(nprop):
            b.step(1)
            ms, nl = b.step_timing()
            ms_tot += ms
            nl_tot += nl
        bps, _ = chs[0].step_bytes()
        avg = ms_tot / 1e3 / max(nl_tot, 1)
        ws = nch * chain_state_bytes(chs[0])
        achieved = nch * bps / avg / 1e9
        kern = "k_step<float>" if prec == g.FP32_ACC64 else "k_step<double>"
        out.append({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "kernel": kern,
                    "traffic": traffic_bytes(kern, nch, ppt, nt, bt),
                    "workload": f"{nch} chains of 32^3, M=2048, "
                                f"{'FP32 recursion / FP64 sums' if prec else 'FP64'}",
                    "working_set_bytes": ws, "pairs_per_thread": ppt, "lanes": lanes,
                    "nontemporal": nt, "block_threads": bt,
                    "avg_round_us": avg * 1e6, "bytes_per_round": nch * bps,
                    "rounds_timed": nl_tot})
        b.close()
        del chs
        torch.cuda.empty_cache()
    return out


def small_configs(g, torch, dev):
    """The two small workloads, FP64 (the oracle's figures for them are in
    the cpu_baseline leg):
    4^3, M = 256, beta = 20, uniform-sphere starts and proposals, seeds 1-3,
    two sweeps each (three chains in one batch, LDS-resident kernel: the
    shape a new batch of chains that fit LDS starts in);
    16^3, M = 1024, T = 0.05, ferromagnet with floor(0.1 N) = 409 random
    sites (seed 42), cap proposals of 0.3 rad: 256 proposals timed, the ten
    sweeps (40 960 proposals) extrapolated."""
    out = {}
    chs = [g.Chain(g.Params(L=4, M=256, beta=20.0, precision=g.FP64, seed=s, chain_id=0),
                   device=dev) for s in (1, 2, 3)]
    for ch in chs:
        ch.init_spins(g.INIT_RANDOM)
    b = g.Batch(chs)
    assert b.tuning()[0] == 0
    b.step(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.sweep(2)
    e1.record(b.stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    b.close()
    svu = 64 * 7 * 128
    out["4cubed_M256_fp64"] = {
        "chains": 3, "proposals_per_chain": 128, "wall_s": dt,
        "proposals_per_s": 3 * 128 / dt, "svu_per_s": 3 * 128 * svu / dt}
    ch = g.Chain(g.Params(L=16, M=1024, beta=20.0, precision=g.FP64, seed=42, chain_id=0,
                          proposal=g.PROPOSE_CONE, cone_angle=0.3), device=dev)
    ch.init_spins(g.INIT_FM_PLUS_RANDOM, 0.1)
    b = g.Batch([ch])
    b.autotune(8)
    form = b.form()
    b.step(2)
    torch.cuda.synchronize()
    n2 = 256
    e0.record(b.stream)
    b.step(n2)
    e1.record(b.stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    b.close()
    svu = 4096 * 7 * 512
    out["16cubed_M1024_fp64_cone"] = {
        "step_launches": ("one persistent launch per proposal on one compute die "
                          f"({form['persistent']} working blocks)" if form["persistent"]
                          else "one launch per Chebyshev step"),
        "proposals_timed": n2, "proposals_per_s": n2 / dt, "svu_per_s": n2 * svu / dt,
        "ten_sweeps_s": 40960 * dt / n2, "ten_sweeps_note": "extrapolated from the timed proposals"}
    return out


def mixed_batch(g, torch, dev, n_prop: int = 2, step_granular: bool = True):
    """One 64^3 chain (M = 4096) and eight 32^3 chains (M = 2048) in one
    batch, FP32 recursion, T = 0.05, uniform-sphere starts from seed 11.
    Step-granular schedule (default): in the 2048 step rounds of one 64^3
    proposal each 32^3 chain makes two proposals, each started as soon as
    its last one is reconstructed; lock-step: every chain one proposal per
    batched proposal, the 32^3 chains idle for the second half.  n_prop
    timed windows after one warm-up window."""
    chs = [g.Chain(g.Params(L=64, M=4096, beta=20.0, precision=g.FP32_ACC64, seed=11,
                            chain_id=0), device=dev)]
    for c in range(8):
        chs.append(g.Chain(g.Params(L=32, M=2048, beta=20.0, precision=g.FP32_ACC64, seed=11,
                                    chain_id=1 + c), device=dev))
    for ch in chs:
        ch.init_spins(g.INIT_RANDOM)
    b = g.Batch(chs)
    b.autotune(256)
    ppt, lanes = b.tuning()
    nt, bt = b.form()["nontemporal"], b.block_threads()
    b.set_schedule(step_granular)
    b.step(1)
    torch.cuda.synchronize()
    c0 = [ch.get_counter() for ch in chs]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_tot, nl_tot = 0.0, 0
    e0.record(b.stream)
    for _ in range(n_prop):
        b.step(1)
        ms, nl = b.step_timing()
        ms_tot += ms
        nl_tot += nl
    e1.record(b.stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    props = [ch.get_counter() - c for ch, c in zip(chs, c0)]
    svu = sum(p * ch.p.L ** 3 * 7 * (ch.p.M // 2) for p, ch in zip(props, chs))
    moved = 0.0
    for p, ch in zip(props, chs):
        bps, ns = ch.step_bytes()
        moved += p * bps * ns
    b.close()
    rec = {"workload": "one 64^3 chain (M=4096) + eight 32^3 chains (M=2048), FP32 recursion, "
                       "T=0.05, uniform-sphere starts (seed 11)",
           "schedule": "step-granular" if step_granular else "lock-step",
           "windows": n_prop, "proposals": {"64^3": props[0], "32^3_each": props[1]},
           "ms_per_window": 1e3 * dt / n_prop,
           "svu_per_s": svu / dt, "mc_spin_updates_per_s": sum(props) / dt,
           "pairs_per_thread": ppt, "lanes": lanes, "nontemporal": nt, "block_threads": bt}
    # step kernel: algorithmic bytes of every step taken over the step time
    # (step-granular: the whole window, reconstructions of the 32^3 chains
    # included; lock-step: the step launches)
    rec["step_kernel"] = {"rounds": nl_tot, "avg_round_us": 1e3 * ms_tot / max(nl_tot, 1),
                          "achieved_GBs": moved / (ms_tot / 1e3) / 1e9,
                          "frac": moved / (ms_tot / 1e3) / 1e9 / HBM_PEAK_GBS}
    return rec


# serving mixes: lattice sizes, their probabilities, default arrival rate (1/s;
# None: set from the offered load, a fraction of a stated capacity in svu/s)
SERVING_MIXES = {
    # small chains: L <= 8 on the LDS-resident kernel, 12 and 16 multi-block
    "small": ((4, 6, 8, 12, 16), (0.3, 0.25, 0.25, 0.15, 0.05), 6.0),
    # the serving workload's sizes whose sweeps finish within minutes on one GPU
    "large": ((8, 16, 24, 32), (0.4, 0.3, 0.2, 0.1), 0.3),
    # the full serving workload: L uniform in {8, 16, 24, 32, 48}
    "full": ((8, 16, 24, 32, 48), (0.2, 0.2, 0.2, 0.2, 0.2), None),
}


def serving_request_svu(L: int) -> float:
    """Work of one request of lattice size L in site-vector updates: N
    proposals per sweep, N * 7 * M/2 per proposal, M = min(2048, 64 L);
    2 sweeps for L <= 24, 1 above."""
    N, M = L ** 3, min(2048, 64 * L)
    return (2 if L <= 24 else 1) * N * N * 7 * (M // 2)


def serving(g, seconds: float, mix: str = "small", seed: int = 2024, emit: bool = True,
            load: float = 1.0, capacity_svu: float = 0.0, drain_s: float = 1e9):
    """Continuous-batching serving run: Poisson arrivals (seeded) of chains
    from a mix of lattice sizes, M = min(2048, 64 L) (K the next power of
    two), T uniform in [0.02, 0.2], FP32 recursion, 2 sweeps per request for
    L <= 24 and 1 above; arrivals stop after `seconds`, then the engine
    drains for at most `drain_s` seconds and the requests still running are
    cancelled and reported as unfinished (their sweep latency is at least
    the time they ran).  A mix without a fixed rate arrives at `load` x
    `capacity_svu` / (mean svu per request).  Prints a progress line every
    30 s and one JSON line with the per-sweep latency percentiles overall and
    per L, the queueing delay and the throughput, and returns that record;
    with emit=False (a leg of the default benchmark) the progress lines go to
    stderr and nothing else is printed."""
    import numpy as np
    sizes, probs, rate = SERVING_MIXES[mix]
    mean_svu = sum(p * serving_request_svu(Lk) for Lk, p in zip(sizes, probs))
    if rate is None:
        if capacity_svu <= 0:
            raise ValueError(f"mix {mix} needs a capacity (svu/s) to set its arrival rate")
        rate = load * capacity_svu / mean_svu
    rng = np.random.default_rng(seed)
    eng = g.Engine(0, hbm_budget_bytes=32 << 30, max_slots=64)
    t0 = time.perf_counter()
    t_next, k, meta, t_print = rng.exponential(1.0 / rate), 0, {}, 30.0
    admitted_at = {}

    def progress(now):
        st = eng.status()
        print(json.dumps({"mode": "serving_progress", "t_s": round(now, 1), "submitted": k,
                          **st}), file=sys.stdout if emit else sys.stderr, flush=True)

    while True:
        now = time.perf_counter() - t0
        if now >= seconds:
            break
        if now >= t_print:
            progress(now)
            t_print += 30.0
        if now >= t_next:
            Lk = int(rng.choice(sizes, p=probs))
            Mk = min(2048, 64 * Lk)
            Kk = 1 << (Mk - 1).bit_length()
            T = float(rng.uniform(0.02, 0.2))
            rid = eng.submit(g.Params(L=Lk, M=Mk, K=Kk, beta=1.0 / T, precision=g.FP32_ACC64,
                                      seed=seed, chain_id=k), init=g.INIT_RANDOM,
                             nsweeps=2 if Lk <= 24 else 1)
            meta[rid] = Lk
            k += 1
            t_next += rng.exponential(1.0 / rate)
        else:
            time.sleep(min(0.01, max(0.0, t_next - now)))
    t_drain = time.perf_counter()
    unfinished = []
    while True:   # drain, reporting progress, for at most drain_s
        try:
            eng.drain(min(30.0, max(1.0, drain_s - (time.perf_counter() - t_drain))))
            break
        except g.GfmcError as e:
            if e.status != g.GFMC_EBUSY:
                raise
            progress(time.perf_counter() - t0)
            if time.perf_counter() - t_drain >= drain_s:
                done_ids = set()
                for rid in meta:
                    try:
                        eng.cancel(rid)
                        unfinished.append(rid)
                    except g.GfmcError:
                        done_ids.add(rid)
                eng.drain(120.0)
                break
    wall = time.perf_counter() - t0
    res = eng.poll(1 << 16)
    lat, ids = eng.sweep_latencies()
    eng.close()
    ok = [r for r in res if r.status == 0]
    props = sum(r.proposals for r in res)
    svu = sum(r.proposals * (r.L ** 3) * 7 * (r.M // 2) for r in res)
    per_L = {}
    for Lk in sizes:
        sel = np.array([meta.get(int(i)) == Lk for i in ids], dtype=bool)
        rec_L = {"requests": sum(1 for v in meta.values() if v == Lk)}
        if sel.any():
            rec_L.update({"p50_s": float(np.percentile(lat[sel], 50)),
                          "p99_s": float(np.percentile(lat[sel], 99)), "sweeps": int(sel.sum())})
        cut = [r for r in res if r.status == g.GFMC_ECANCELED and meta.get(r.request_id) == Lk]
        if cut:
            # a request cancelled at the drain limit: its open sweep had run at least this long
            rec_L["unfinished"] = len(cut)
            rec_L["unfinished_sweep_lower_bound_s"] = [
                round(r.t_done - (r.t_first_sweep if r.t_first_sweep >= 0 else r.t_admit), 1)
                for r in cut if r.t_admit >= 0]
            rec_L["unfinished_queued"] = sum(1 for r in cut if r.t_admit < 0)
            # the rate they ran at: proposals done in their open sweep, and the
            # sweep time that rate projects (N proposals per sweep)
            rec_L["unfinished_open_sweep_proposals"] = [
                int(r.proposals % (Lk ** 3)) for r in cut if r.t_admit >= 0]
            rec_L["unfinished_projected_sweep_s"] = [
                round((r.t_done - (r.t_first_sweep if r.t_first_sweep >= 0 else r.t_admit)) *
                      Lk ** 3 / max(1, r.proposals % (Lk ** 3)), 1)
                for r in cut if r.t_admit >= 0]
        per_L[str(Lk)] = rec_L
    wait = np.array([r.t_admit - r.t_submit for r in res if r.t_admit >= 0])
    rec = {
        "mode": "serving", "mix": mix, "requests": k, "completed": len(ok),
        "unfinished_at_drain_limit": len(unfinished),
        "arrival_rate_per_s": rate, "arrival_window_s": seconds,
        "drain_limit_s": drain_s if drain_s < 1e8 else None, "wall_s": wall,
        "offered_load": ({"fraction_of_capacity": load, "capacity_svu_per_s": capacity_svu,
                          "mean_request_svu": mean_svu}
                         if SERVING_MIXES[mix][2] is None else None),
        "sweep_latency_s": ({"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99))} if len(lat) else {}) |
                           {"per_L": per_L, "sweeps": int(len(lat))},
        "queue_wait_s": ({"p50": float(np.percentile(wait, 50)),
                          "p99": float(np.percentile(wait, 99))} if len(wait) else {}),
        "mc_spin_updates_per_s": props / wall, "svu_per_s": svu / wall,
        "config": {"workload": f"Poisson arrivals ({rate:.4g}/s), L in {sorted(set(sizes))} w.p. "
                               f"{probs}, M = min(2048, 64 L), T ~ U[0.02, 0.2], FP32 recursion, "
                               "2 sweeps per request for L <= 24 and 1 above, 32 GiB budget, "
                               "64 slots"}}
    if emit:
        print(json.dumps(rec), flush=True)
    return rec


def copy_sweep(torch):
    """Bandwidth of a plain device copy (read + write) and of a read-only
    reduction (torch sum) over working sets of 16 MiB .. 2 GiB: below the
    256 MB last-level cache the repeated passes are served partly from it."""
    for mib in (16, 32, 64, 128, 192, 256, 384, 512, 1024, 2048):
        n = (mib << 20) // 8                  # float32 elements per copy buffer (half the span)
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        reps = max(5, (4096 // mib))
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(reps):
            dst.copy_(src)
        c1.record()
        torch.cuda.synchronize()
        s = c0.elapsed_time(c1) / 1e3
        del src, dst
        # read-only: one buffer spanning the whole working set
        buf = torch.ones(2 * n, dtype=torch.float32, device="cuda:0")
        out = torch.empty((), dtype=torch.float32, device="cuda:0")
        for _ in range(3):
            torch.sum(buf, dim=(0,), out=out)
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record()
        for _ in range(reps):
            torch.sum(buf, dim=(0,), out=out)
        r1.record()
        torch.cuda.synchronize()
        sr = r0.elapsed_time(r1) / 1e3
        print(json.dumps({"mode": "copy_sweep", "span_MiB": mib, "reps": reps,
                          "copy_GBs": reps * 2 * 4 * n / s / 1e9,
                          "read_only_GBs": reps * 8 * n / sr / 1e9}), flush=True)
        del buf, out


def physics(g, torch, warm: int = 50, sweeps: int = 200):
    """Magnetization |m| against temperature (the paper's validation: M = 256,
    mu = 0): ten temperatures per lattice size, ferromagnetic starts, FP64
    recursion, one batch per size; `warm` sweeps discarded, then the mean of
    |m| over `sweeps` sweeps with the error from 10 blocks, and the
    acceptance rate."""
    import numpy as np
    temps = [0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.3, 0.5, 1.0]
    for Lk in (4, 6, 8):
        t0 = time.perf_counter()
        chs = [g.Chain(g.Params(L=Lk, M=256, beta=1.0 / T, mu=0.0, precision=g.FP64, seed=2013,
                                chain_id=i)) for i, T in enumerate(temps)]
        for ch in chs:
            ch.init_spins(g.INIT_FM)
        b = g.Batch(chs)
        b.autotune(4)
        b.sweep(warm)
        mags, acc = b.sweep(sweeps)
        b.close()
        blocks = mags.reshape(len(temps), 10, -1).mean(axis=2)
        print(json.dumps({
            "mode": "physics", "L": Lk, "M": 256, "mu": 0.0, "warmup_sweeps": warm,
            "sweeps": sweeps, "T": temps, "m_mean": [float(v) for v in mags.mean(axis=1)],
            "m_err": [float(v) for v in blocks.std(axis=1, ddof=1) / np.sqrt(10)],
            "acceptance": [float(a) / (sweeps * Lk ** 3) for a in acc],
            "wall_s": time.perf_counter() - t0}), flush=True)


def fp32_accuracy(g, sites: int = 16, sizes=(2, 4, 6, 8, 10, 12, 16, 24, 32, 48, 64),
                  moments=(256, 512, 1024, 2048, 4096, 8192), betas=(20.0, 50.0)):
    """Error of the FP32 recursion (FP64 sums) against the FP64 recursion, per
    lattice size L and moment count M: max |d mu| over the 7x7 moments and
    max / mean |d Delta S| at each beta, over `sites` seeded sites and moves
    (uniform random spins).  The FP64 path itself matches the oracle to
    1e-12 / 1e-10.  Cells outside the FP32 range the library accepts are
    measured with the guard lifted for this purpose only (EINVAL otherwise)."""
    import numpy as np
    import synth
    for Lk in sizes:
        th, ph = synth.random_angles(Lk ** 3, 5)
        for Mk in moments:
            try:
                c32 = g.Chain(g.Params(L=Lk, M=Mk, beta=betas[0], precision=g.FP32_ACC64,
                                       fp32_unvalidated=1))
            except g.GfmcError as e:
                print(json.dumps({"mode": "fp32_accuracy", "L": Lk, "M": Mk, "error": str(e)}),
                      flush=True)
                continue
            c64 = g.Chain(g.Params(L=Lk, M=Mk, beta=betas[0], precision=g.FP64))
            for c in (c32, c64):
                c.set_spins(th, ph)
            rng = np.random.default_rng(Lk * 100003 + Mk)
            moves = []
            for _ in range(sites):
                o = int(rng.integers(Lk ** 3))
                moves.append((o, float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))))
            dmu = max(float(np.abs(c32.moments(o) - c64.moments(o)).max()) for o, _, _ in moves)
            rec = {"mode": "fp32_accuracy", "L": Lk, "M": Mk, "sites": sites, "max_dmu": dmu}
            for b in betas:
                for c in (c32, c64):
                    c.set_params(1.0, b, 0.0)
                dds = [abs(c32.delta_seff(o, tn, pn) - c64.delta_seff(o, tn, pn)) for o, tn, pn in moves]
                rec[f"max_dds_beta{b:g}"] = max(dds)
                rec[f"mean_dds_beta{b:g}"] = float(np.mean(dds))
            c32.close()
            c64.close()
            print(json.dumps(rec), flush=True)


def chain_sweep(g, torch):
    """Step-kernel time and algorithmic bandwidth of 32^3, M = 2048 batches of
    8..128 chains (FP32 and FP64), both launch shapes, one or two lanes, 256-
    or 512-thread blocks: shows where the chains' data stops fitting the 256 MB
    last-level cache."""
    for prec in (g.FP32_ACC64, g.FP64):
        for nch in (8, 16, 32, 64, 128):
            chs = [g.Chain(g.Params(L=L, M=M, beta=20.0, precision=prec, seed=SEED, chain_id=c))
                   for c in range(nch)]
            for c in chs:
                c.init_spins(g.INIT_RANDOM)
            b = g.Batch(chs)
            bps, _ = chs[0].step_bytes()
            for bt, ppt, lanes in ((256, 1, 1), (256, 2, 1), (256, 1, 2), (256, 2, 2),
                                   (512, 1, 1), (512, 1, 2)):
                b.set_lanes(lanes)
                b.set_block_threads(bt)
                b.set_tuning(ppt)
                b.step(1)
                b.step(2)
                ms, nl = b.step_timing()
                us = ms * 1e3 / nl
                print(json.dumps({"mode": "chain_sweep", "precision": "f32" if prec else "f64",
                                  "chains": nch, "pairs_per_thread": ppt, "block_threads": bt,
                                  "lanes": b.tuning()[1], "avg_round_us": us,
                                  "achieved_GBs": nch * bps / (us * 1e-6) / 1e9,
                                  "bytes_per_round": nch * bps}), flush=True)
            b.close()
            del chs
            torch.cuda.empty_cache()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU (chains shard across GPUs by process); "
                                   "--gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_probe:
        n = 1 << 28                       # 2^28 float32 = 1 GiB per buffer
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "dispatches": 3}), flush=True)
        return
    if args.copy_sweep:
        copy_sweep(torch)
        return
    import paper_1303_6016_amd as g
    import synth
    if args.serving > 0:
        serving(g, args.serving, args.serving_mix, load=args.serving_load,
                capacity_svu=args.serving_capacity, drain_s=args.serving_drain)
        return
    if args.chain_sweep:
        chain_sweep(g, torch)
        return
    if args.physics:
        physics(g, torch)
        return
    if args.fp32_accuracy:
        fp32_accuracy(g)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    temps = synth.temperature_ladder(NCHAIN, T_LO, T_HI)
    chains = []
    for c in range(NCHAIN):
        p = g.Params(L=L, M=M, beta=1.0 / temps[c], mu=0.0, precision=g.FP32_ACC64,
                     seed=SEED, chain_id=c)
        ch = g.Chain(p, device=dev)
        ch.init_spins(g.INIT_RANDOM)
        chains.append(ch)
    batch = g.Batch(chains)
    tune(batch, args.tuning)
    ppt, lanes = batch.tuning()
    nt = batch.form()["nontemporal"]
    bt = batch.block_threads()
    if args.graph:
        batch.use_graph(True)
    stream = batch.stream
    bytes_per_step, nsteps = chains[0].step_bytes()
    N = L ** 3
    svu_per_prop = N * 7 * (M // 2)

    for _ in range(args.warmup):
        batch.step(1)
    torch.cuda.synchronize()

    # timed region: K steps, per-step events for the latency distribution
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    step_ms_total, launches_total = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        batch.step(1)
        ms, nl = batch.step_timing()
        step_ms_total += ms
        launches_total += nl
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]) / 1e3
    total_s = float(lat.sum())
    ms_per_step = 1e3 * total_s / args.steps
    value = args.steps * NCHAIN * svu_per_prop / total_s

    # dominant kernel: the Chebyshev step, averaged over every step round in the
    # timed region (a round is one step of all 64 chains: one launch of
    # k_step, or with two lanes one launch per lane, the two running at once)
    avg_round_s = step_ms_total / 1e3 / max(launches_total, 1)
    bytes_per_round = NCHAIN * bytes_per_step
    achieved = bytes_per_round / avg_round_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes("k_step<float>", NCHAIN, ppt, nt, bt),
            "kernel": "k_step<float>", "lanes": lanes,
            "round": "one Chebyshev step of all chains" +
                     (": two concurrent k_step launches, one per lane" if lanes == 2 else
                      ": one k_step launch"),
            "avg_round_us": avg_round_s * 1e6, "bytes_per_round": bytes_per_round}

    # the device's streaming ceilings, measured live with the library's own
    # streaming kernel: two reads + one write per item (the step kernel's mix)
    # over buffers well above the 256 MB last-level cache (HBM), and over
    # 64 MiB buffers (cache-resident, the regime of this batch)
    ceil_hbm = g.stream_bandwidth(3, 1 << 30, 10)
    ceil_llc = g.stream_bandwidth(3, 64 << 20, 20)
    ws = NCHAIN * chain_state_bytes(chains[0])
    roof["working_set_bytes"] = ws
    roof["regime"] = ("last-level-cache resident: the chains' vectors and spinors "
                      f"({ws / 1e6:.0f} MB) fit the 256 MB Infinity Cache, so this fraction is "
                      "read against the HBM peak but served partly from the cache; the HBM "
                      "figures are the roofline_hbm_regime records")
    roof["ceiling_2r1w_hbm_GBs"] = ceil_hbm
    roof["ceiling_2r1w_llc_GBs"] = ceil_llc
    roof["frac_of_llc_ceiling"] = achieved / ceil_llc

    out = {
        "metric": "Chebyshev site-vector updates/s + MC spin updates/s at 32^3; p50/p99 sweep latency",
        "value": value, "unit": "svu/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "32^3 lattice x 64 chains, M=2048, FP32 recursion / FP64 moment "
                               "sums, T=0.02..0.2 t, uniform-sphere starts (seed 7)",
                   "L": L, "M": M, "chains": NCHAIN, "graph": bool(args.graph),
                   "pairs_per_thread": ppt, "lanes": lanes, "nontemporal": nt,
                   "block_threads": bt},
        "mc_spin_updates_per_s": args.steps * NCHAIN / total_s,
        "step_latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "sweep_latency_s": {"p50": float(np.percentile(lat, 50)) * N,
                            "p99": float(np.percentile(lat, 99)) * N,
                            "note": "extrapolated: one sweep = N batched steps"},
        "wall_s": wall,
        "roofline": roof,
    }
    # the other form of the same work: each proposal replayed as one captured
    # HIP graph (the headline above launches directly)
    if not args.graph:
        try:
            batch.use_graph(True)
            batch.step(1)
            torch.cuda.synchronize()
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ng = 3
            g0.record(stream)
            batch.step(ng)
            g1.record(stream)
            torch.cuda.synchronize()
            gms = g0.elapsed_time(g1) / ng
            out["graph_replay"] = {"ms_per_step": gms, "direct_ms_per_step": ms_per_step,
                                   "value": NCHAIN * svu_per_prop / (gms / 1e3),
                                   "speedup_over_direct": ms_per_step / gms}
            batch.use_graph(False)
        except Exception as e:   # the headline stands on its own
            out["graph_replay"] = {"error": str(e)}

    if args.pair:
        note("pair form")
        # the same workload with the {o, v} start-vector pair (2 vectors per proposal)
        pch = []
        for c in range(NCHAIN):
            p = g.Params(L=L, M=M, beta=1.0 / temps[c], mu=0.0, precision=g.FP32_ACC64,
                         seed=SEED, chain_id=c, vectors=g.VECTORS_OV)
            ch = g.Chain(p, device=dev)
            ch.init_spins(g.INIT_RANDOM)
            pch.append(ch)
        pb = g.Batch(pch)
        tune(pb, args.pair_tuning)
        pppt, plan = pb.tuning()
        pb.step(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nps = max(4, args.steps // 2)
        ms_tot, nl_tot = 0.0, 0
        e0.record(pb.stream)
        for _ in range(nps):
            pb.step(1)
            ms, nl = pb.step_timing()
            ms_tot += ms
            nl_tot += nl
        e1.record(pb.stream)
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3
        pbytes, psteps = pch[0].step_bytes()
        # algorithmic bytes of one proposal's step launches: one step per launch
        # reads the two stored values and the spinor of every site and writes one
        # value (40 B/site FP32); the two-step shape (3) runs step 1 so, then per
        # launch reads both slots and the spinor once and writes both slots
        # (48 B/site for two steps: 1.2 x one step's bytes)
        if pppt == 3:
            prop_bytes = NCHAIN * pbytes * (1 + 1.2 * (psteps // 2))
            kern = "k_step_ov2<float>"
            rnd = "step 1, then two Chebyshev steps of all chains per k_step_ov2 launch"
        else:
            prop_bytes = NCHAIN * pbytes * psteps
            kern = "k_step_ov<float>"
            rnd = "one Chebyshev step of all chains"
        achieved = prop_bytes * nps / (ms_tot / 1e3) / 1e9
        pavg = ms_tot / 1e3 / max(nl_tot, 1)
        out["pair_form"] = {
            "mc_spin_updates_per_s": nps * NCHAIN / dt,
            "svu_per_s": nps * NCHAIN * N * 2 * (M // 2) / dt,
            "ms_per_step": 1e3 * dt / nps, "pairs_per_thread": pppt, "lanes": plan,
            "roofline": {"bound": "hbm", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic_bytes(kern, NCHAIN, pppt),
                         "kernel": kern, "lanes": plan, "round": rnd,
                         "avg_round_us": pavg * 1e6,
                         "bytes_per_round": prop_bytes * nps / max(nl_tot, 1)}}
        pb.close()
        del pch

    if args.stored_hops:
        note("stored hopping rows")
        # A/B: the same workload with stored hopping rows instead of recomputation
        hch = []
        for c in range(NCHAIN):
            p = g.Params(L=L, M=M, beta=1.0 / temps[c], mu=0.0, precision=g.FP32_ACC64,
                         seed=SEED, chain_id=c, hoppings=g.HOP_STORED)
            ch = g.Chain(p, device=dev)
            ch.init_spins(g.INIT_RANDOM)
            hch.append(ch)
        hb = g.Batch(hch)
        hb.set_tuning(ppt)
        hb.set_lanes(lanes)
        hb.step(1)
        torch.cuda.synchronize()
        nps = max(2, args.steps // 4)
        ms_tot, nl_tot = 0.0, 0
        for _ in range(nps):
            hb.step(1)
            ms, nl = hb.step_timing()
            ms_tot += ms
            nl_tot += nl
        hbytes, _ = hch[0].step_bytes()
        havg = ms_tot / 1e3 / max(nl_tot, 1)
        out["stored_hoppings_ab"] = {
            "kernel": "k_step<float> with stored rows", "pairs_per_thread": ppt, "lanes": lanes,
            "avg_round_us": havg * 1e6, "bytes_per_round": NCHAIN * hbytes,
            "achieved_GBs": NCHAIN * hbytes / havg / 1e9,
            "slowdown_vs_recompute": havg / avg_round_s,
            "traffic": traffic_bytes("k_step<float> stored rows", NCHAIN, ppt)}
        hb.close()
        del hch

    if not args.no_fp64_single:
        note("plain FP64 single chain")
        p = g.Params(L=L, M=M, beta=1.0 / T_LO, precision=g.FP64, seed=SEED, chain_id=0)
        ch = g.Chain(p, device=dev)
        ch.init_spins(g.INIT_RANDOM)
        ch.step()
        torch.cuda.synchronize()
        n1 = 4
        t1 = time.perf_counter()
        for _ in range(n1):
            ch.step()
        torch.cuda.synchronize()
        d1 = time.perf_counter() - t1
        out["fp64_single_chain"] = {"mc_spin_updates_per_s": n1 / d1,
                                    "svu_per_s": n1 * svu_per_prop / d1,
                                    "proposals": n1}
        out["batched_vs_fp64_single_speedup"] = out["mc_spin_updates_per_s"] / (n1 / d1)

    def leg(name, fn):
        # a secondary leg that raises is recorded; the headline line still prints
        try:
            return fn()
        except Exception as e:
            note(f"{name} failed: {e}")
            return {"error": str(e)}

    if args.hbm:
        note("HBM-regime step kernel (128 x 32^3 FP32, 64 x 32^3 FP64)")
        hr = leg("HBM regime", lambda: hbm_regime(g, torch, dev, args.tuning))
        out["roofline_hbm_regime"] = hr
        if isinstance(hr, list):
            for r in hr:
                r["ceiling_2r1w_hbm_GBs"] = roof["ceiling_2r1w_hbm_GBs"]
                r["frac_of_hbm_ceiling"] = r["achieved"] / roof["ceiling_2r1w_hbm_GBs"]
    if args.mixed:
        note("64^3 + 8 x 32^3 batch")
        out["mixed_64cubed_plus_8x32cubed"] = leg("mixed batch", lambda: mixed_batch(g, torch, dev))
    if args.small:
        note("4^3 and 16^3 workloads")
        out["small_configs"] = leg("small workloads", lambda: small_configs(g, torch, dev))
    batch.close()
    if args.serving_leg:
        # the metric's p50/p99 sweep latency under continuous batching; every
        # batch of the other legs is closed (their streams released), so the
        # engine's three streams and torch's get a hardware queue each
        note("serving (30 s of Poisson arrivals)")
        try:
            sv = serving(g, 30.0, "small", emit=False)
            out["serving"] = {
                "mix": "small", "workload": sv["config"]["workload"],
                "arrival_window_s": sv["arrival_window_s"], "requests": sv["requests"],
                "completed": sv["completed"], "sweep_latency_s": sv["sweep_latency_s"],
                "queue_wait_s": sv["queue_wait_s"],
                "mc_spin_updates_per_s": sv["mc_spin_updates_per_s"]}
        except Exception as e:   # the headline must still be reported
            note(f"serving leg failed: {e}")
            out["serving"] = {"error": str(e)}

    if not args.no_cpu_baseline:
        note("oracle on the host cores")
        out["cpu_baseline"] = leg("oracle baseline", cpu_baseline)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
