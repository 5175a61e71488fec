"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/gfmc.h declares, and validates parameters without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gfmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gfmc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1303_6016_amd as g
    L = g.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(g.EXPORTS)
    assert L.gfmc_version().decode().startswith("gfmc")


def _bytes(**kw):
    import paper_1303_6016_amd as g
    return g.gfmc_workspace_bytes(g.Params(**kw))


@pytest.mark.parametrize("kw", [dict(L=3), dict(L=0), dict(L=4, M=7), dict(L=4, M=256, K=300),
                                dict(L=4, M=512, K=256), dict(L=4, beta=0.0), dict(L=4, t=-1.0),
                                dict(L=4, scale_b=0.1), dict(L=4, scale_a=1.0),
                                dict(L=4, proposal=1, cone_angle=0.0), dict(L=4, precision=5),
                                dict(L=4, M=16384), dict(L=4, vectors=1, hoppings=1),
                                dict(L=4, vectors=3), dict(L=4, vectors=2, hoppings=1),
                                dict(L=4, hoppings=3), dict(L=4, kernel=-1),
                                dict(L=4, proposal=7), dict(L=4, precision=-2**31)])
def test_invalid_parameters_are_rejected(kw):
    import paper_1303_6016_amd as g
    with pytest.raises(g.GfmcError) as e:
        _bytes(**kw)
    assert e.value.status == g.GFMC_EINVAL


def test_workspace_size_follows_layout():
    # the bipartite layout stores 7 complex values per site in the recursion precision
    b64 = _bytes(L=32, M=2048, precision=0)
    b32 = _bytes(L=32, M=2048, precision=1)
    N = 32 ** 3
    assert b64 - b32 >= 7 * N * 8 + 2 * N * 4 * 2
    assert b64 > 7 * N * 16


def test_null_handles_and_bad_arguments_are_rejected_on_the_host():
    # these return before any device call, so they run without a GPU
    import paper_1303_6016_amd as g
    L = g.lib()
    i32, d = ctypes.c_int32(), ctypes.c_double()
    buf = (ctypes.c_double * 8)()
    EINVAL = g.GFMC_EINVAL
    assert L.gfmc_batch_set_lanes(None, 2) == EINVAL
    assert L.gfmc_batch_get_tuning(None, ctypes.byref(i32), ctypes.byref(i32)) == EINVAL
    assert L.gfmc_batch_set_tuning(None, 1) == EINVAL
    assert L.gfmc_batch_autotune(None, 4, ctypes.byref(i32)) == EINVAL
    assert L.gfmc_batch_step(None, 1, None, None) == EINVAL
    assert L.gfmc_mixed_moments(None, 0, 1.0, 1.0, buf) == EINVAL
    assert L.gfmc_pair_moments(None, 0, 1.0, 1.0, buf) == EINVAL
    assert L.gfmc_delta_seff(None, 0, 1.0, 1.0, ctypes.byref(d), ctypes.byref(d)) == EINVAL
    assert L.gfmc_engine_submit(None, None, 0, 0.0, 1, None) == EINVAL
    sz, h = ctypes.c_size_t(), ctypes.c_void_p()
    assert L.gfmc_batch_workspace_bytes(None, 0, ctypes.byref(sz)) == EINVAL
    assert L.gfmc_batch_create(None, 0, None, 0, None, ctypes.byref(h)) == EINVAL
    with pytest.raises(g.GfmcError) as e:
        g.Batch([])
    assert e.value.status == EINVAL
    assert L.gfmc_chain_destroy(None) == g.GFMC_OK and L.gfmc_batch_destroy(None) == g.GFMC_OK
    assert L.gfmc_last_error()
    # status codes are taken as plain integers: any value has a text
    assert L.gfmc_status_string(EINVAL) == b"invalid argument"
    for v in (1, 7, -7, 2 ** 31 - 1, -2 ** 31):
        assert L.gfmc_status_string(v) == b"unknown status"


# The validated range of the FP32 recursion (include/gfmc.h, gfmc_precision):
# just inside and just outside its edges in M and in beta t.
FP32_EDGES = [(4, 1024), (6, 1024), (8, 4096), (12, 4096), (16, 8192), (32, 8192), (64, 8192)]


@pytest.mark.parametrize("L,M", FP32_EDGES)
def test_fp32_guard_edges_in_moment_count(L, M):
    import paper_1303_6016_amd as g
    assert _bytes(L=L, M=M, precision=1, beta=50.0) > 0
    if M < 8192:
        with pytest.raises(g.GfmcError) as e:
            _bytes(L=L, M=M + 2, K=2 * M, precision=1, beta=20.0)
        assert e.value.status == g.GFMC_EINVAL and "validated" in str(e.value)
        # FP64 has no such limit; FP32 outside the range is available for measuring its error
        assert _bytes(L=L, M=M + 2, K=2 * M, precision=0) > 0
        assert _bytes(L=L, M=M + 2, K=2 * M, precision=1, fp32_unvalidated=1) > 0


def test_fp32_guard_refuses_the_smallest_lattice():
    import paper_1303_6016_amd as g
    with pytest.raises(g.GfmcError) as e:
        _bytes(L=2, M=32, precision=1)
    assert e.value.status == g.GFMC_EINVAL
    assert _bytes(L=2, M=32, precision=0) > 0
    assert _bytes(L=2, M=32, precision=1, fp32_unvalidated=1) > 0


def test_fp32_guard_edge_in_beta():
    import paper_1303_6016_amd as g
    assert _bytes(L=32, M=2048, precision=1, beta=1.0 / 0.02) > 0
    assert _bytes(L=32, M=2048, precision=1, beta=25.0, t=2.0) > 0
    for kw in (dict(beta=50.001), dict(beta=26.0, t=2.0)):
        with pytest.raises(g.GfmcError) as e:
            _bytes(L=32, M=2048, precision=1, **kw)
        assert e.value.status == g.GFMC_EINVAL
    assert _bytes(L=32, M=2048, precision=0, beta=1000.0) > 0
    with pytest.raises(g.GfmcError):
        _bytes(L=32, M=2048, precision=1, fp32_unvalidated=2)
