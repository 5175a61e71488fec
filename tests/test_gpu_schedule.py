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
    assert g.lib().gfmc_batch_set_schedule(b.h, 2) == g.GFMC_EINVAL
    b.close()
    for i, sp in enumerate(specs):
        ch = mk(i, *sp)
        for _ in range([4, 5][i]):
            ch.step()
        th, ph = ch.get_spins()
        gth, gph = chs[i].get_spins()
        assert np.array_equal(gth, th) and np.array_equal(gph, ph)


@pytest.mark.parametrize("L,M,prec", [(16, 256, 0), (12, 128, 1), (10, 64, 0), (24, 64, 1),
                                      (14, 128, 1), (20, 64, 0)])
def test_lone_chain_persistent_run_equals_step_launches(g, L, M, prec):
    # A lone chain that fits one compute die runs all M/2 steps of a proposal
    # in one persistent launch; the same chain beside another one in a batch
    # runs one launch per step.  Same step arithmetic, so the vectors agree
    # bit for bit; the persistent kernel's blocks are half the size, so its
    # block partial sums group the sites differently and Delta S agrees to
    # rounding of the FP64 sums.  Decisions and spins must be equal, and the
    # moments must match the oracle's.
    import oracle
    import synth
    p = g.Params(L=L, M=M, beta=20.0, precision=prec, seed=5, chain_id=2)
    probe = g.Chain(p)
    pb = g.Batch([probe])
    # the lone chain takes the persistent path, with blocks of 64 threads while
    # that gives at most 16 blocks, else of 128 or 256 (at most 32 blocks)
    expected_blocks = {10: 8, 12: 14, 14: 11, 16: 16, 20: 32, 24: 27}[L]
    assert pb.form()["persistent"] == expected_blocks
    pb.close()
    lone = g.Chain(p)
    th, ph = synth.random_angles(L ** 3, 3)
    lone.set_spins(th, ph)
    mu = lone.moments(17)
    ref = oracle.moments(oracle.Model(L=L, M=M, beta=20.0, seed=5, chain_id=2), th, ph, 17)
    assert np.abs(mu - ref).max() < (1e-12 if prec == 0 else 1e-5)
    recs = [lone.step() for _ in range(4)]
    a = g.Chain(p)
    a.set_spins(th, ph)
    other = g.Chain(g.Params(L=L, M=M, beta=5.0, precision=prec, seed=9))
    b = g.Batch([a, other])
    b.set_tuning(1)
    assert b.form()["persistent"] == 0
    brecs = b.step(4, records=True)
    b.close()
    for q in range(4):
        assert brecs[q][0].site == recs[q].site
        assert abs(brecs[q][0].dseff - recs[q].dseff) <= 1e-11 * max(1.0, abs(recs[q].dseff))
        assert brecs[q][0].accepted == recs[q].accepted
    t1, p1 = lone.get_spins()
    t2, p2 = a.get_spins()
    assert np.array_equal(t1, t2) and np.array_equal(p1, p2)


def test_nontemporal_steps_do_not_change_results(g):
    # non-temporal loads and stores change only how the caches keep the lines
    def run(nt):
        chs = [g.Chain(g.Params(L=L, M=64, beta=10.0, precision=1, seed=12, chain_id=i))
               for i, L in enumerate((12, 16))]
        for c in chs:
            c.init_spins(g.INIT_RANDOM)
        b = g.Batch(chs)
        b.set_tuning(1)
        b.set_nontemporal(nt)
        assert b.form()["nontemporal"] == int(nt)
        recs = b.step(3, records=True)
        b.close()
        return [(r.site, r.dseff, r.accepted) for row in recs for r in row], \
               [c.get_spins() for c in chs]
    r0, s0 = run(False)
    r1, s1 = run(True)
    assert r0 == r1
    for (a, b_), (c, d) in zip(s0, s1):
        assert np.array_equal(a, c) and np.array_equal(b_, d)


@pytest.mark.parametrize("prec,ppt,lanes", [(0, 1, 1), (1, 2, 2), (1, 1, 2)])
def test_512_thread_blocks_match_256(g, prec, ppt, lanes):
    # The launched step kernel with 512-thread blocks forms the same vectors
    # (same per-site arithmetic) and groups the block partial sums over twice
    # the sites: decisions, sites and spins equal the 256-thread run's, Delta S
    # agrees to rounding of the FP64 sums and matches the oracle.  12^3 and
    # 10^3 leave a ragged last block.
    import oracle
    import synth
    specs = [(12, 64, 10.0), (10, 128, 5.0), (16, 64, 20.0)]

    def run(bt):
        chs = []
        for i, (L, M, beta) in enumerate(specs):
            ch = g.Chain(g.Params(L=L, M=M, beta=beta, precision=prec, seed=41, chain_id=i))
            th, ph = synth.random_angles(L ** 3, 70 + i)
            ch.set_spins(th, ph)
            chs.append(ch)
        b = g.Batch(chs)
        b.set_tuning(ppt)
        b.set_lanes(lanes)
        b.set_block_threads(bt)
        assert b.block_threads() == bt and b.tuning() == (ppt, lanes)
        spins0 = [c.get_spins() for c in chs]
        recs = b.step(3, records=True)
        b.close()
        return recs, [c.get_spins() for c in chs], spins0
    r256, s256, spins0 = run(256)
    r512, s512, _ = run(512)
    for q in range(3):
        for i in range(len(specs)):
            a, c = r256[q][i], r512[q][i]
            assert (a.site, a.u, a.accepted) == (c.site, c.u, c.accepted)
            assert abs(a.dseff - c.dseff) <= 1e-11 * max(1.0, abs(a.dseff))
    for (t1, p1), (t2, p2) in zip(s256, s512):
        assert np.array_equal(t1, t2) and np.array_equal(p1, p2)
    tol = 1e-10 if prec == 0 else 2e-5
    for i, (L, M, beta) in enumerate(specs):
        m = oracle.Model(L=L, M=M, beta=beta, seed=41, chain_id=i)
        th, ph = spins0[i]
        r = r512[0][i]
        ref = oracle.delta_seff(m, th, ph, r.site, r.theta_new, r.phi_new)
        assert abs(r.dseff - ref) < tol


def test_block_threads_validation(g):
    ch = g.Chain(g.Params(L=12, M=64, precision=0, seed=1))
    b = g.Batch([ch])
    for bad in (0, 64, 128, 1024):
        with pytest.raises(g.GfmcError) as e:
            b.set_block_threads(bad)
        assert e.value.status == g.GFMC_EINVAL
    b.close()
    for kw in ({"vectors": 1}, {"hoppings": 1}):
        c = g.Chain(g.Params(L=12, M=64, precision=0, seed=1, **kw))
        bb = g.Batch([c])
        with pytest.raises(g.GfmcError) as e:
            bb.set_block_threads(512)
        assert e.value.status == g.GFMC_EINVAL
        assert bb.block_threads() == 256
        bb.close()
