"""Serving engine on the GPU: continuous batching of uneven chains gives each
request the same result as running it alone; admission by slots and HBM
budget; cancellation."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_6016_amd as g
    g.lib()
    return g


SPECS = [  # L, M, T, precision, init, nsweeps
    (4, 128, 0.05, 0, 0, 2),
    (6, 64, 0.2, 1, 0, 1),
    (4, 256, 0.1, 1, 2, 1),
    (2, 32, 0.02, 0, 1, 3),
    (6, 128, 0.15, 0, 0, 1),
]


def params(g, i, spec):
    L, M, T, prec, _, _ = spec
    return g.Params(L=L, M=M, beta=1.0 / T, precision=prec, seed=2024, chain_id=i)


def test_engine_results_equal_alone_runs(g):
    eng = g.Engine(0, hbm_budget_bytes=256 << 20, max_slots=3)
    ids = []
    for i, spec in enumerate(SPECS):
        ids.append(eng.submit(params(g, i, spec), init=spec[4], frac=0.1, nsweeps=spec[5]))
        time.sleep(0.01)   # staggered arrivals join running work
    eng.drain(600)
    res = {r.request_id: r for r in eng.poll()}
    lat, lat_ids = eng.sweep_latencies()
    assert len(lat) == sum(s[5] for s in SPECS) and np.all(lat > 0)
    st = eng.status()
    assert st["running"] == 0 and st["queued"] == 0 and st["bytes"] == 0
    eng.close()
    for i, spec in enumerate(SPECS):
        r = res[ids[i]]
        assert r.status == 0 and r.sweeps == spec[5]
        ch = g.Chain(params(g, i, spec))
        ch.init_spins(spec[4], 0.1)
        mag, acc = ch.sweep(spec[5])
        print(f"request {i}: L={spec[0]} M={spec[1]} accepted {r.accepted} alone {acc} "
              f"|m| {r.magnetization:.12f} alone {mag[-1]:.12f}", flush=True)
        assert r.proposals == spec[5] * spec[0] ** 3
        assert r.accepted == acc
        assert r.magnetization == mag[-1]
        assert abs(r.magnetization_mean - mag.mean()) < 1e-15
        assert r.t_submit <= r.t_admit <= r.t_first_sweep <= r.t_done


def test_engine_budget_and_cancel(g):
    p_big = g.Params(L=32, M=2048)
    eng = g.Engine(0, hbm_budget_bytes=8 << 20, max_slots=2)
    with pytest.raises(g.GfmcError) as e:
        eng.submit(p_big)
    assert e.value.status == g.GFMC_EBUSY
    long_id = eng.submit(g.Params(L=8, M=256, seed=1), nsweeps=1000)
    queued_id = eng.submit(g.Params(L=8, M=256, seed=2), nsweeps=1000)
    third = eng.submit(g.Params(L=8, M=256, seed=3), nsweeps=1000)   # waits for a slot
    # poll the engine's state (bounded) until both slots are taken
    deadline = time.monotonic() + 60.0
    while eng.status()["running"] < 2 and time.monotonic() < deadline:
        time.sleep(0.005)
    st = eng.status()
    assert st["running"] == 2 and st["queued"] == 1, st
    eng.cancel(third)
    eng.cancel(long_id)
    eng.cancel(queued_id)
    eng.drain(120)
    res = {r.request_id: r for r in eng.poll()}
    assert {long_id, queued_id, third} <= set(res)
    assert all(res[i].status == g.GFMC_ECANCELED for i in (long_id, queued_id, third))
    with pytest.raises(g.GfmcError):
        eng.cancel(long_id)
    eng.close()



def _wait_status(eng, pred, timeout=60.0):
    deadline = time.monotonic() + timeout
    st = eng.status()
    while not pred(st) and time.monotonic() < deadline:
        time.sleep(0.005)
        st = eng.status()
    return st


def test_engine_admits_smaller_requests_past_one_that_does_not_fit(g):
    # budget = A + B - 256 bytes: with A running, B (no larger than A) does
    # not fit, C does; C goes in ahead of B, and B goes in once A has left
    # (into A's place: the budget is carved first-fit)
    pa = g.Params(L=16, M=1024, seed=1)
    pb = g.Params(L=12, M=512, seed=2)
    pc = g.Params(L=4, M=64, seed=3)
    al = lambda n: (n + 255) // 256 * 256
    wa, wb, wc = (al(g.gfmc_workspace_bytes(p)) for p in (pa, pb, pc))
    assert wa >= wb > wc + 256
    eng = g.Engine(0, hbm_budget_bytes=wa + wb - 256, max_slots=4)
    ida = eng.submit(pa, nsweeps=100000)
    st = _wait_status(eng, lambda st: st["running"] == 1)
    assert st["running"] == 1, st
    idb = eng.submit(pb, nsweeps=100000)
    idc = eng.submit(pc, nsweeps=100000)
    st = _wait_status(eng, lambda st: st["running"] == 2)
    assert st["running"] == 2 and st["queued"] == 1, st   # A and C run, B waits
    eng.cancel(ida)
    st = _wait_status(eng, lambda st: st["queued"] == 0 and st["running"] == 2)
    assert st["running"] == 2 and st["queued"] == 0, st   # B took A's place
    eng.cancel(idb)
    eng.cancel(idc)
    eng.drain(120)
    res = {r.request_id: r for r in eng.poll()}
    assert all(res[i].status == g.GFMC_ECANCELED for i in (ida, idb, idc))
    assert res[idc].t_admit < res[idb].t_admit   # C was admitted before B
    eng.close()


def test_engine_holds_admission_for_a_request_that_waited(g):
    # A request that has waited 10 s without fitting holds admission: a small
    # request submitted after that waits behind it (no starvation of large
    # requests by a stream of small ones).  Same sizes as above.
    pa = g.Params(L=16, M=1024, seed=1)
    pb = g.Params(L=12, M=512, seed=2)
    pc = g.Params(L=4, M=64, seed=3)
    al = lambda n: (n + 255) // 256 * 256
    wa, wb, wc = (al(g.gfmc_workspace_bytes(p)) for p in (pa, pb, pc))
    eng = g.Engine(0, hbm_budget_bytes=wa + wb - 256, max_slots=4)
    ida = eng.submit(pa, nsweeps=100000)
    st = _wait_status(eng, lambda st: st["running"] == 1)
    assert st["running"] == 1, st
    idb = eng.submit(pb, nsweeps=100000)
    time.sleep(10.5)
    idc = eng.submit(pc, nsweeps=100000)
    time.sleep(1.0)
    st = eng.status()
    assert st["running"] == 1 and st["queued"] == 2, st   # C waits behind B
    eng.cancel(ida)   # B goes in, then C
    st = _wait_status(eng, lambda st: st["running"] == 3 or (st["running"] == 2 and st["queued"] == 0))
    assert st["queued"] == 0, st
    for i in (idb, idc):
        eng.cancel(i)
    eng.drain(120)
    res = {r.request_id: r for r in eng.poll()}
    assert res[idb].t_admit <= res[idc].t_admit
    eng.close()

MIXED = [  # L, M, T, precision: LDS-resident (L <= 10 FP32, L <= 8 FP64) and multi-block chains
    (4, 128, 0.05, 1),
    (10, 64, 0.1, 0),
    (12, 64, 0.2, 1),
    (10, 64, 0.15, 1),
    (16, 64, 0.05, 1),
    (6, 64, 0.02, 0),
]


def test_engine_mixed_kernel_shapes_equal_alone_runs(g):
    # small chains run several proposals per iteration beside the multi-block
    # ones; each stops exactly at its sweep boundaries, so |m| per sweep and
    # the accepted count equal the alone run's
    eng = g.Engine(0, hbm_budget_bytes=1 << 30, max_slots=8)
    ids = [eng.submit(g.Params(L=L, M=M, beta=1.0 / T, precision=prec, seed=99, chain_id=i),
                      init=g.INIT_RANDOM, nsweeps=2)
           for i, (L, M, T, prec) in enumerate(MIXED)]
    eng.drain(600)
    res = {r.request_id: r for r in eng.poll()}
    eng.close()
    for i, (L, M, T, prec) in enumerate(MIXED):
        r = res[ids[i]]
        ch = g.Chain(g.Params(L=L, M=M, beta=1.0 / T, precision=prec, seed=99, chain_id=i))
        ch.init_spins(g.INIT_RANDOM)
        mag, acc = ch.sweep(2)
        print(f"mixed request {i}: L={L} prec={prec} accepted {r.accepted} alone {acc} "
              f"|m| {r.magnetization:.12f} alone {mag[-1]:.12f}", flush=True)
        assert r.status == 0 and r.sweeps == 2 and r.proposals == 2 * L ** 3
        assert r.accepted == acc
        assert r.magnetization == mag[-1]
        assert abs(r.magnetization_mean - mag.mean()) < 1e-15


def test_engine_rejects_negative_caps(g):
    import ctypes
    eng = g.Engine(0, hbm_budget_bytes=8 << 20, max_slots=1)
    L = g.lib()
    n = ctypes.c_int32(7)
    out = (g.Result * 1)()
    sec = (ctypes.c_double * 1)()
    assert L.gfmc_engine_poll(eng.h, out, -1, ctypes.byref(n)) == g.GFMC_EINVAL
    assert L.gfmc_engine_sweep_latencies(eng.h, sec, None, -1, ctypes.byref(n)) == g.GFMC_EINVAL
    assert n.value == 7
    eng.close()
