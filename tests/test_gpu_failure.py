"""Failure detection on the GPU: a chain whose state is corrupted is flagged
and rejects its proposals, and the other chains of its batch are unaffected.

Non-finite angles are written into one chain's workspace on the device
(gfmc_chain_device_angles gives their address; gfmc_set_spins would refuse
them).  Every proposal of that chain then has a non-finite Delta S_eff: it must
be rejected, even when the decision is forced, and counted
(gfmc_chain_nonfinite), while the two other chains of the batch take exactly
the trajectories they take in a batch of their own (same kernels and block
tables: bit for bit).
"""
import ctypes
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_6016_amd as g
    g.lib()
    return g


def _poke(dev_ptr: int, values: np.ndarray):
    """Host to device copy through the HIP runtime the library runs on (by its
    soname, which resolves to the copy already loaded in the process)."""
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipDeviceSynchronize.argtypes = []
    src = np.ascontiguousarray(values, dtype=np.float64)
    assert hip.hipDeviceSynchronize() == 0
    assert hip.hipMemcpy(dev_ptr, src.ctypes.data, src.nbytes, 1) == 0   # host to device


SPECS = [(10, 64), (12, 64), (14, 64)]   # multi-block chains, FP64


def _chain(g, i, L, M):
    ch = g.Chain(g.Params(L=L, M=M, beta=10.0, precision=0, seed=31, chain_id=i))
    th, ph = synth.random_angles(L ** 3, 60 + i)
    ch.set_spins(th, ph)
    return ch


def test_nonfinite_state_is_flagged_and_spares_the_other_chains(g):
    nprop = 4
    healthy = [_chain(g, i, *SPECS[i]) for i in (0, 2)]
    hb = g.Batch(healthy)
    hb.set_tuning(1)
    hb.set_lanes(1)
    hrecs = hb.step(nprop, records=True)
    hb.close()
    alone = {}
    for j, i in enumerate((0, 2)):
        alone[i] = ([hrecs[q][j] for q in range(nprop)], healthy[j].get_spins())
        assert healthy[j].nonfinite() == 0
    chs = [_chain(g, i, L, M) for i, (L, M) in enumerate(SPECS)]
    L1 = SPECS[1][0]
    th_ptr, _ = chs[1].device_angles()
    _poke(th_ptr, np.full(L1 ** 3, np.nan))
    b = g.Batch(chs)
    b.set_tuning(1)
    b.set_lanes(1)
    recs = b.step(nprop, records=True)
    b.close()
    for q in range(nprop):
        r = recs[q][1]
        assert not math.isfinite(r.dseff) and r.accepted == 0 and r.own == 0
    assert chs[1].nonfinite() == nprop
    for i in (0, 2):
        ref_recs, (th, ph) = alone[i]
        for q in range(nprop):
            r, a = recs[q][i], ref_recs[q]
            assert (r.site, r.accepted, r.dseff) == (a.site, a.accepted, a.dseff)
        gth, gph = chs[i].get_spins()
        assert np.array_equal(gth, th) and np.array_equal(gph, ph)
        assert chs[i].nonfinite() == 0
    # a forced acceptance must not take a non-finite proposal either
    r = chs[1].step(force=1)
    assert r.accepted == 0 and not math.isfinite(r.dseff)
    assert chs[1].nonfinite() == nprop + 1
