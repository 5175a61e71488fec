"""Step-granular batch schedule on the GPU (gfmc_batch_set_schedule).

Chains of different moment counts share the step launches; each chain
restarts its next proposal as soon as its last one is reconstructed, so in a
window of nprop x M_max/2 step rounds a chain of M makes nprop x M_max / M
proposals.  Every chain must end exactly where the same chain run alone for
that many proposals ends: spins bit for bit, the proposal counter and the
accepted count (both paths run the multi-block step kernel with one site
pair per thread, so the sums are formed in the same order).
"""
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


# (L, M, T): multi-block chains (too large for the LDS-resident kernel)
SPECS = [(12, 128, 0.05), (12, 64, 0.1), (14, 32, 0.2), (12, 64, 0.02), (16, 128, 0.15),
         (12, 32, 0.07)]


def _chain(g, i, L, M, T, prec, vectors):
    ch = g.Chain(g.Params(L=L, M=M, beta=1.0 / T, precision=prec, seed=77, chain_id=i,
                          vectors=vectors))
    ch.init_spins(g.INIT_RANDOM)
    return ch


def _alone(g, i, L, M, T, prec, vectors, nprop):
    ch = _chain(g, i, L, M, T, prec, vectors)
    assert ch.__class__ is g.Chain
    for _ in range(nprop):
        ch.step()
    th, ph = ch.get_spins()
    return th, ph, ch.get_counter()


@pytest.mark.parametrize("prec,vectors,lanes,graph", [(1, 0, 1, False), (0, 0, 2, False),
                                                      (1, 1, 2, False), (1, 0, 1, True)])
def test_step_granular_batch_equals_alone_runs(g, prec, vectors, lanes, graph):
    nwin = 2
    chs = [_chain(g, i, L, M, T, prec, vectors) for i, (L, M, T) in enumerate(SPECS)]
    b = g.Batch(chs)
    b.set_tuning(1)
    b.set_lanes(lanes)
    b.set_schedule(True)
    if graph:
        b.use_graph(True)
        for _ in range(nwin):
            b.step(1)
    else:
        b.step(nwin)
    ms, rounds = b.step_timing()
    mmax = max(M for _, M, _ in SPECS)
    got = [(c.get_spins(), c.get_counter()) for c in chs]
    b.close()
    for i, (L, M, T) in enumerate(SPECS):
        nprop = nwin * mmax // M
        th, ph, ctr = _alone(g, i, L, M, T, prec, vectors, nprop)
        (gth, gph), gctr = got[i]
        print(f"chain {i}: L={L} M={M} proposals {gctr} (alone {ctr})", flush=True)
        assert gctr == ctr == nprop
        assert np.array_equal(gth, th) and np.array_equal(gph, ph)
    if not graph:
        assert rounds == nwin * mmax // 2 and ms > 0


def test_step_granular_uneven_counts_and_validation(g):
    # M = 128 and 80 (K = 128): a window of nprop x 64 rounds holds nprop
    # proposals of the first chain and floor(nprop x 64 / 40) of the second
    specs = [(12, 128, 0.05), (12, 80, 0.1)]

    def mk(i, L, M, T):
        ch = g.Chain(g.Params(L=L, M=M, K=128, beta=1.0 / T, precision=1, seed=78, chain_id=i))
        ch.init_spins(g.INIT_RANDOM)
        return ch
    chs = [mk(i, *sp) for i, sp in enumerate(specs)]
    b = g.Batch(chs)
    b.set_tuning(1)
    b.set_schedule(True)
    with pytest.raises(g.GfmcError) as e:
        b.step(1, records=True)
    assert e.value.status == g.GFMC_EINVAL
    b.step(3)   # 192 rounds: 3 proposals of M = 128, 4 of M = 80 (32 rounds idle)
    assert [c.get_counter() for c in chs] == [3, 4]
    b.set_schedule(False)
    b.step(1)   # lock-step: one more each
    assert [c.get_counter() for c in chs] == [4, 5]
    with pytest.raises(g.GfmcError):
        b.set_schedule(2)
    b.close()
    for i, sp in enumerate(specs):
        ch = mk(i, *sp)
        for _ in range([4, 5][i]):
            ch.step()
        th, ph = ch.get_spins()
        gth, gph = chs[i].get_spins()
        assert np.array_equal(gth, th) and np.array_equal(gph, ph)
