"""The allocation-free entry point gfmc_delta_seff_static against the chain
entry point gfmc_delta_seff (GPU).

Two or more calls in a row on one device share the library's static scratch
array; each later call is smaller than the one before, so a stale tail of an
earlier call's buffers would show.  On the LDS-resident chains both entry
points run the same kernels in the same launch shape, so the values must agree
bit for bit.  The chain entry point runs a lone multi-block chain on the
persistent kernel, whose blocks are half the size of the step launches the
static entry point makes: the vectors agree bit for bit, the block sums group
the sites differently, and the values agree to the parity bar (1e-10 in FP64,
2e-5 in FP32).
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (L, M, precision, beta, start vectors): a multi-block chain first, then
# LDS-resident ones, each call smaller than the one before
CASES = [(12, 256, 1, 20.0, 0), (8, 512, 0, 20.0, 0), (6, 128, 1, 10.0, 1), (4, 64, 0, 5.0, 0)]


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_6016_amd as g
    g.lib()
    return g


def _static(g, p, dth, dph, o, tn, pn, out, stream):
    cp = p.c()
    return g.lib().gfmc_delta_seff_static(
        ctypes.byref(cp), ctypes.c_void_p(dth.data_ptr()), ctypes.c_void_p(dph.data_ptr()), o,
        tn, pn, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8),
        ctypes.c_void_p(stream.cuda_stream))


def test_static_entry_matches_chain_entry(g):
    import torch
    import synth
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    for L, M, prec, beta, vec in CASES:
        p = g.Params(L=L, M=M, beta=beta, precision=prec, seed=3, vectors=vec)
        th, ph = synth.random_angles(L ** 3, 17 + L)
        ch = g.Chain(p)
        ch.set_spins(th, ph)
        dth = torch.tensor(th, dtype=torch.float64, device=dev)
        dph = torch.tensor(ph, dtype=torch.float64, device=dev)
        rng = np.random.default_rng(L * 7 + M)
        tol = 1e-10 if prec == 0 else 2e-5
        for _ in range(3):
            o = int(rng.integers(L ** 3))
            tn, pn = float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))
            ref, rtop = ch.delta_seff(o, tn, pn, with_phase_top=True)
            out = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
            assert _static(g, p, dth, dph, o, tn, pn, out, st) == g.GFMC_OK, \
                g.lib().gfmc_last_error().decode()
            torch.cuda.synchronize()
            got, top = out.cpu().numpy()
            print(f"L={L} M={M} prec={prec} vectors={vec} site={o}: dS {got:.12f} "
                  f"chain {ref:.12f}", flush=True)
            assert abs(got - ref) < tol and abs(top - rtop) < tol
            if L <= 8:   # LDS-resident on both paths
                assert got == ref and top == rtop
        # the inputs are read only
        assert np.array_equal(dth.cpu().numpy(), th) and np.array_equal(dph.cpu().numpy(), ph)
        ch.close()


def test_static_entry_rejects_oversized_and_invalid(g):
    import torch
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    big = g.Params(L=64, M=4096, precision=0)
    t = torch.zeros(64 ** 3, dtype=torch.float64, device=dev)
    assert _static(g, big, t, t, 0, 1.0, 1.0, out, st) == g.GFMC_EINVAL
    assert b"scratch" in g.lib().gfmc_last_error()
    small = g.Params(L=4, M=64)
    t4 = torch.zeros(64, dtype=torch.float64, device=dev)
    assert _static(g, small, t4, t4, 64, 1.0, 1.0, out, st) == g.GFMC_EINVAL
    assert _static(g, small, t4, t4, 0, float("nan"), 1.0, out, st) == g.GFMC_EINVAL
