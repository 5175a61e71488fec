"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (absolute; |mu| <= 1):
  moments     FP64 1e-12, FP32 recursion / FP64 sums 1e-5
  Delta S     FP64 1e-10, FP32 2e-5
  The FP32 bounds hold for M <= 1024 on every lattice and at the benchmark
  sizes (32^3 with M = 2048, 64^3 with M = 4096); on small lattices the FP32
  error grows with M beyond them (bench.py --fp32-accuracy measures it).
  RNG, sites, Metropolis draws: bit-exact; new angles within a few ulp
  (device and host libm may round acos/atan2 differently).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FP64_MU, FP32_MU = 1e-12, 1e-5
FP64_DS, FP32_DS = 1e-10, 2e-5


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_6016_amd as g
    g.lib()
    return g


def make(g, L, M, prec=0, seed=0, chain_id=0, **kw):
    p = g.Params(L=L, M=M, precision=prec, seed=seed, chain_id=chain_id, **kw)
    m = oracle.Model(L=L, M=M, seed=seed, chain_id=chain_id,
                     **{k: v for k, v in kw.items() if k in ("t", "beta", "mu", "K")})
    if "proposal" in kw:
        m.proposal = kw["proposal"]
    if "cone_angle" in kw:
        m.cone = kw["cone_angle"]
    if "kernel" in kw:
        m.kernel = kw["kernel"]
    if kw.get("lorentz_lambda"):
        m.lam = kw["lorentz_lambda"]
    return g.Chain(p), m


# ----------------------------------------------------------------- moments --
@pytest.mark.parametrize("L,M,seed,sites", [(2, 32, 1, [0, 5]), (4, 256, 2, [0, 1, 37, 63]),
                                            (6, 128, 3, [0, 100, 215]), (8, 256, 4, [3, 511])])
@pytest.mark.parametrize("prec", [0, 1])
def test_moments_small(g, L, M, seed, sites, prec):
    if prec == 1 and L < 4:   # outside the FP32 recursion's validated range
        with pytest.raises(g.GfmcError) as e:
            make(g, L, M, prec)
        assert e.value.status == g.GFMC_EINVAL
        return
    ch, m = make(g, L, M, prec)
    th, ph = synth.random_angles(m.N, seed)
    ch.set_spins(th, ph)
    tol = FP64_MU if prec == 0 else FP32_MU
    for o in sites:
        got = ch.moments(o)
        ref = oracle.moments(m, th, ph, o)
        err = np.abs(got - ref).max()
        print(f"L={L} M={M} prec={prec} site={o} max|dmu|={err:.2e}", flush=True)
        assert err < tol


def test_moments_16cubed_ferro_plus_random(g):
    ch, m = make(g, 16, 1024, 0, seed=42)
    ch.init_spins(g.INIT_FM_PLUS_RANDOM, 0.1)
    th, ph = ch.get_spins()
    tho, pho = oracle.init_spins(m, 2, 0.1)
    assert np.array_equal(th != 0, tho != 0) and (th != 0).sum() == 409
    assert np.array_equal(ph, pho)
    assert np.abs(th - tho).max() <= 4 * np.spacing(np.pi)
    for o in (0, 2049):
        err = np.abs(ch.moments(o) - oracle.moments(m, th, ph, o)).max()
        print(f"16^3 M=1024 site={o} max|dmu|={err:.2e}", flush=True)
        assert err < FP64_MU


@pytest.mark.parametrize("prec,tol", [(0, FP64_MU), (1, FP32_MU)])
def test_moments_32cubed_full_size_sampled(g, prec, tol):
    # the workload size of the benchmark: one sampled site, oracle one by one
    ch, m = make(g, 32, 2048, prec, seed=7, chain_id=3)
    ch.init_spins(g.INIT_RANDOM)
    th, ph = ch.get_spins()
    o = 12345
    ref = oracle.moments(m, th, ph, o)
    err = np.abs(ch.moments(o) - ref).max()
    print(f"32^3 M=2048 prec={prec} max|dmu|={err:.2e}", flush=True)
    assert err < tol


def test_moment_invariants_on_device(g):
    ch, m = make(g, 8, 128, 0)
    th, ph = synth.random_angles(m.N, 12)
    ch.set_spins(th, ph)
    mu = ch.moments(77)
    assert np.abs(mu[0] - np.eye(7)).max() == 0
    assert np.abs(mu - mu.conj().transpose(0, 2, 1)).max() < 1e-14
    assert np.abs(mu).max() <= 1 + 1e-12
    assert np.all(mu[1::2, 0, 0] == 0) and np.all(mu[0::2, 0, 1:] == 0)


# ----------------------------------------------------------------- Delta S --
# includes the extremes M = 2 (mu_0 and mu_1 only), M = 4, and K = 8192 nodes
# zero-padded over M = 64 on the 2^3 lattice (doubled bonds)
@pytest.mark.parametrize("L,M,K,beta", [(4, 256, 0, 20.0), (6, 256, 512, 5.0), (8, 512, 0, 20.0),
                                        (4, 64, 0, 0.5), (4, 2, 0, 5.0), (6, 4, 0, 5.0),
                                        (2, 64, 8192, 20.0)])
@pytest.mark.parametrize("prec", [0, 1])
def test_delta_seff(g, L, M, K, beta, prec):
    if prec == 1 and L < 4:   # outside the FP32 recursion's validated range
        with pytest.raises(g.GfmcError) as e:
            make(g, L, M, prec, beta=beta, K=K)
        assert e.value.status == g.GFMC_EINVAL
        return
    ch, m = make(g, L, M, prec, beta=beta, K=K)
    th, ph = synth.random_angles(m.N, 5)
    ch.set_spins(th, ph)
    tol = FP64_DS if prec == 0 else FP32_DS
    rng = np.random.default_rng(1)
    for _ in range(3):
        o = int(rng.integers(m.N))
        tn, pn = float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))
        got, top = ch.delta_seff(o, tn, pn, with_phase_top=True)
        ref, rtop = oracle.delta_seff(m, th, ph, o, tn, pn, with_phase_top=True)
        print(f"L={L} M={M} K={K} beta={beta} prec={prec} dS={ref:.6f} err={got - ref:.2e}",
              flush=True)
        assert abs(got - ref) < tol
        # top-edge phase: a diagnostic amplified by 1/sin(th) at the band edge
        assert abs(top - rtop) < (1e-8 if prec == 0 else 1e-2)


def test_delta_seff_largest_moment_count(g):
    # M = K = 8192, the largest the library accepts: the reconstruction block
    # holds 8192 nodes in LDS.  FP64 on 4^3 against the oracle; the FP32
    # recursion at this M lies outside its validated range on 4^3 (EINVAL) and
    # inside it on 32^3, where it must meet the FP32 bound at the range's
    # largest beta t = 50.
    m = oracle.Model(L=4, M=8192, beta=20.0)
    th, ph = synth.random_angles(m.N, 5)
    ref, rtop = oracle.delta_seff(m, th, ph, 3, 1.0, 2.0, with_phase_top=True)
    ch, _ = make(g, 4, 8192, 0, beta=20.0)
    ch.set_spins(th, ph)
    got, top = ch.delta_seff(3, 1.0, 2.0, with_phase_top=True)
    print(f"4^3 M=K=8192 FP64 dS={ref:.6f} err={got - ref:.2e} top={top:.2e}", flush=True)
    assert abs(got - ref) < FP64_DS and abs(top - rtop) < 1e-8
    with pytest.raises(g.GfmcError) as e:
        make(g, 4, 8192, 1, beta=20.0)
    assert e.value.status == g.GFMC_EINVAL
    m32 = oracle.Model(L=32, M=8192, beta=50.0, seed=2, chain_id=5)
    th, ph = synth.random_angles(m32.N, 6)
    ref = oracle.delta_seff(m32, th, ph, 1234, 1.0, 2.0)
    ch, _ = make(g, 32, 8192, 1, beta=50.0, seed=2, chain_id=5)
    ch.set_spins(th, ph)
    got = ch.delta_seff(1234, 1.0, 2.0)
    print(f"32^3 M=K=8192 FP32 beta=50 dS={ref:.6f} err={got - ref:.2e}", flush=True)
    assert abs(got - ref) < FP32_DS


def test_delta_seff_lorentz_and_identity(g):
    ch, m = make(g, 4, 128, 0, kernel=1, lorentz_lambda=4.0)
    th, ph = synth.random_angles(m.N, 9)
    ch.set_spins(th, ph)
    got = ch.delta_seff(10, 1.0, 2.0)
    assert abs(got - oracle.delta_seff(m, th, ph, 10, 1.0, 2.0)) < FP64_DS
    assert ch.delta_seff(10, th[10], ph[10]) == 0.0


# ---------------------------------------------------- teacher-forced chains --
def run_forced(g, ch, m, th, ph, nprop, prec):
    tol = FP64_DS if prec == 0 else FP32_DS
    forced = 0
    for idx in range(nprop):
        ro = oracle.step(m, th, ph, idx)
        rg = ch.step(force=ro.accepted)
        assert rg.index == ro.index == idx
        assert rg.site == ro.site and rg.u == ro.u
        assert abs(rg.theta_new - ro.theta_new) <= 4 * np.spacing(max(ro.theta_new, 1.0))
        assert abs(rg.phi_new - ro.phi_new) <= 4 * np.spacing(max(ro.phi_new, 1.0))
        assert abs(rg.dseff - ro.dseff) < tol, (idx, rg.dseff, ro.dseff)
        near = abs(math.log(ro.u) + ro.dseff) < 10 * tol if ro.u > 0 else False
        if rg.own != ro.own:
            assert near, (idx, rg.dseff, ro.dseff, ro.u)
            forced += 1
        assert rg.accepted == ro.accepted
    gth, gph = ch.get_spins()
    assert np.abs(gth - th).max() < 1e-13 and np.abs(gph - ph).max() < 1e-13
    return forced


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_trajectory_4cubed_two_sweeps(g, seed):
    # 4^3, M = 256, Jackson, beta = 20, mu = 0, uniform-sphere start and proposals
    ch, m = make(g, 4, 256, 0, seed=seed, beta=20.0)
    ch.init_spins(g.INIT_RANDOM)
    th, ph = oracle.init_spins(m, 0)
    gth, gph = ch.get_spins()
    assert np.array_equal(gph, ph) and np.abs(gth - th).max() <= 4 * np.spacing(np.pi)
    ch.set_spins(th, ph)
    forced = run_forced(g, ch, m, th, ph, 2 * m.N, 0)
    print(f"seed={seed}: 128 proposals, forced decisions {forced}", flush=True)


def test_trajectory_16cubed_prefix_cone(g):
    # 16^3, M = 1024, T = 0.05, FM + 10% random start, cap proposals of 0.3 rad
    ch, m = make(g, 16, 1024, 0, seed=42, beta=20.0, proposal=1, cone_angle=0.3)
    th, ph = oracle.init_spins(m, 2, 0.1)
    ch.set_spins(th, ph)
    forced = run_forced(g, ch, m, th, ph, 12, 0)
    print(f"16^3 prefix: forced {forced}", flush=True)


@pytest.mark.parametrize("L,M,K", [(4, 256, 512), (10, 256, 1024)])
def test_trajectory_lorentz_fine_grid(g, L, M, K):
    # Lorentz kernel (lambda = 4) with a zero-padded K > M energy grid, end to
    # end: draws, Delta S, Metropolis decisions and spin updates; L = 4 runs the
    # LDS-resident kernel, L = 10 the multi-block one
    ch, m = make(g, L, M, 0, seed=8, beta=20.0, K=K, kernel=1, lorentz_lambda=4.0)
    th, ph = oracle.init_spins(m, 0)
    ch.set_spins(th, ph)
    forced = run_forced(g, ch, m, th, ph, 64 if L == 4 else 16, 0)
    print(f"Lorentz L={L} K={K}: forced {forced}", flush=True)


def test_trajectory_fp32(g):
    ch, m = make(g, 8, 256, 1, seed=4, beta=10.0)
    th, ph = synth.random_angles(m.N, 4)
    ch.set_spins(th, ph)
    run_forced(g, ch, m, th, ph, 24, 1)


def test_sweep_matches_oracle(g):
    ch, m = make(g, 4, 128, 0, seed=11, beta=8.0)
    th, ph = synth.random_angles(m.N, 11)
    ch.set_spins(th, ph)
    # oracle trajectory with its own decisions; the device must take the same
    # ones unless an event lands within rounding of the Metropolis threshold
    recs = []
    t2, p2 = th.copy(), ph.copy()
    for idx in range(m.N):
        recs.append(oracle.step(m, t2, p2, idx))
    if any(abs(math.log(r.u) + r.dseff) < 1e-9 for r in recs if r.u > 0):
        pytest.skip("threshold tie in this seed")
    mag, acc = ch.sweep(1)
    gth, gph = ch.get_spins()
    assert acc == sum(r.accepted for r in recs)
    assert np.abs(gth - t2).max() < 1e-13 and np.abs(gph - p2).max() < 1e-13
    assert abs(mag[0] - oracle.magnetization(4, t2, p2)) < 1e-14
    assert ch.get_counter() == m.N


# ------------------------------------------------------------------ batches --
@pytest.mark.parametrize("shape", [0, 1])
def test_batch_results_equal_single_chains(g, shape):
    # shape 0 runs the same LDS-resident kernel as a single chain: bit-identical;
    # shape 1 (multi-block step kernel) differs only in the order of the sums
    specs = [(4, 256, 0.05), (6, 128, 0.1), (8, 256, 0.2), (4, 64, 0.02)]
    def build():
        out = []
        for i, (L, M, T) in enumerate(specs):
            ch, _ = make(g, L, M, 1, seed=100 + i, beta=1.0 / T)
            ch.init_spins(g.INIT_RANDOM)
            out.append(ch)
        return out
    alone = build()
    ref = [[ch.step() for _ in range(6)] for ch in alone]
    mixed = build()
    b = g.Batch(mixed)
    b.set_tuning(shape)
    recs = b.step(6, records=True)
    for q in range(6):
        for i in range(len(specs)):
            r, a = recs[q][i], ref[i][q]
            assert (r.site, r.accepted, r.u) == (a.site, a.accepted, a.u)
            if shape == 0:
                assert r.dseff == a.dseff
            else:
                assert abs(r.dseff - a.dseff) < 1e-5
    b.close()
    for x, y in zip(alone, mixed):
        assert np.array_equal(x.get_spins()[0], y.get_spins()[0])


@pytest.mark.parametrize("ppt", [1, 2])
def test_batch_launch_shapes_agree(g, ppt):
    # moments through a batch with either launch shape equal the single-chain ones
    specs = [(6, 128), (4, 64), (8, 128)]
    alone, mixed = [], []
    for i, (L, M) in enumerate(specs):
        a, m = make(g, L, M, 0, seed=3, chain_id=i, beta=5.0)
        a.init_spins(g.INIT_RANDOM)
        alone.append(a.step())
        b_, _ = make(g, L, M, 0, seed=3, chain_id=i, beta=5.0)
        b_.init_spins(g.INIT_RANDOM)
        mixed.append(b_)
    b = g.Batch(mixed)
    b.set_tuning(ppt)
    recs = b.step(1, records=True)[0]
    for r, a in zip(recs, alone):
        assert r.site == a.site and abs(r.dseff - a.dseff) < 1e-12
    assert b.autotune(4) in (0, 1, 2)
    b.close()


def test_batch_graph_replay_matches_direct(g):
    def build():
        chs = []
        for i in range(3):
            ch, _ = make(g, 6, 128, 0, seed=7, chain_id=i, beta=10.0)
            ch.init_spins(g.INIT_RANDOM)
            chs.append(ch)
        return chs
    a, b = build(), build()
    ba, bb = g.Batch(a), g.Batch(b)
    ba.step(5)
    bb.use_graph(True)
    for _ in range(5):
        bb.step(1)
        bb.chains[0].stream.synchronize()
    ba.close()
    bb.close()
    for x, y in zip(a, b):
        assert np.array_equal(x.get_spins()[0], y.get_spins()[0])
        assert x.get_counter() == y.get_counter() == 5


LANE_SPECS = [(16, 256, 0.05), (12, 128, 0.1), (10, 256, 0.2), (14, 64, 0.02), (10, 128, 0.1)]


def lane_chains(g):
    out = []
    for i, (L, M, T) in enumerate(LANE_SPECS):
        ch, _ = make(g, L, M, 1, seed=21, chain_id=i, beta=1.0 / T)
        ch.init_spins(g.INIT_RANDOM)
        out.append(ch)
    return out


@pytest.mark.parametrize("ppt", [1, 2])
def test_batch_two_lanes_equal_single_chains(g, ppt):
    # multi-block chains of five sizes split over two step lanes (streams):
    # with one site pair per thread the blocks are those of the chain run
    # alone in that shape, so every record is bit-identical; with two the sums
    # are regrouped
    alone = []
    for i, ch in enumerate(lane_chains(g)):
        # each chain beside a partner in one lane: the launched step kernel
        # with the chain's own blocks (a lone chain would run LDS-resident or
        # persistent, whose blocks differ)
        L, M, T = LANE_SPECS[i]
        partner = g.Chain(g.Params(L=L, M=M, beta=1.0 / T, precision=1, seed=99))
        one = g.Batch([ch, partner])
        one.set_tuning(1)
        one.set_lanes(1)
        alone.append([r[0] for r in one.step(3, records=True)])
        one.close()
    mixed = lane_chains(g)
    b = g.Batch(mixed)
    b.set_tuning(ppt)
    b.set_lanes(2)
    assert b.tuning() == (ppt, 2)
    recs = b.step(3, records=True)
    for q in range(3):
        for i in range(len(LANE_SPECS)):
            r, a = recs[q][i], alone[i][q]
            assert (r.site, r.u) == (a.site, a.u)
            if ppt == 1:
                assert (r.accepted, r.dseff) == (a.accepted, a.dseff)
            else:
                assert abs(r.dseff - a.dseff) < 1e-5
    b.close()


def test_lane_arguments(g):
    ch, _ = make(g, 10, 64, 1, seed=3)
    ch.init_spins(g.INIT_RANDOM)
    b = g.Batch([ch])
    assert b.tuning() == (0, 1)     # a new batch of chains that fit LDS starts resident
    b.set_tuning(1)
    for bad in (0, 5):
        with pytest.raises(g.GfmcError) as e:
            b.set_lanes(bad)
        assert e.value.status == g.GFMC_EINVAL
    b.set_lanes(2)                  # a single chain cannot be split: one lane in effect
    assert b.tuning() == (1, 1)
    b.step(1)
    b.close()


def test_batch_graph_replay_with_two_lanes(g):
    # the captured proposal contains both lane streams (fork and join events);
    # every replay, with host synchronisation between them, equals direct launches
    a, b = lane_chains(g), lane_chains(g)
    ba, bb = g.Batch(a), g.Batch(b)
    for x in (ba, bb):
        x.set_tuning(1)
        x.set_lanes(2)
    ba.step(4)
    bb.use_graph(True)
    for _ in range(4):
        bb.step(1)
        bb.chains[0].stream.synchronize()
    assert bb.tuning() == (1, 2)
    ba.close()
    bb.close()
    for x, y in zip(a, b):
        assert np.array_equal(x.get_spins()[0], y.get_spins()[0])
        assert x.get_counter() == y.get_counter() == 4


@pytest.mark.parametrize("shape", [1, 2])
@pytest.mark.parametrize("L,M,prec", [(2, 32, 0), (4, 256, 0), (6, 128, 1)])
def test_step_kernel_shapes_on_small_lattices(g, shape, L, M, prec):
    # the multi-block step kernel on lattices that single chains run resident
    ch, m = make(g, L, M, prec, seed=12, beta=10.0)
    th, ph = synth.random_angles(m.N, 13)
    ch.set_spins(th, ph)
    b = g.Batch([ch])
    b.set_tuning(shape)
    tol = FP64_DS if prec == 0 else FP32_DS
    for idx in range(6):
        ro = oracle.step(m, th, ph, idx)
        rg = b.step(1, force=np.array([ro.accepted]), records=True)[0][0]
        assert rg.site == ro.site and rg.accepted == ro.accepted
        assert abs(rg.dseff - ro.dseff) < tol, (idx, rg.dseff, ro.dseff)
    b.close()


@pytest.mark.parametrize("L,M", [(10, 128), (14, 64)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_multiblock_moments_several_blocks_ragged_tail(g, L, M, prec, tol):
    # single chains of these sizes run the multi-block step kernel: L = 10 has
    # 500 site pairs (2 blocks, the last partial), L = 14 has 1372 (6 blocks)
    ch, m = make(g, L, M, prec)
    th, ph = synth.random_angles(m.N, L + 40)
    ch.set_spins(th, ph)
    for o in (0, m.N // 2 + 3, m.N - 1):
        err = np.abs(ch.moments(o) - oracle.moments(m, th, ph, o)).max()
        print(f"L={L} M={M} prec={prec} site={o}: max|dmu|={err:.1e}", flush=True)
        assert err < tol


@pytest.mark.parametrize("ppt", [1, 2])
def test_multiblock_delta_seff_several_blocks_ragged_tail(g, ppt):
    # both launch shapes through a batch of two ragged-size chains, FP64
    specs = [(14, 64, 0.05), (10, 128, 0.1)]
    chs, ms, sts = [], [], []
    for i, (L, M, T) in enumerate(specs):
        ch, m = make(g, L, M, 0, seed=31, chain_id=i, beta=1.0 / T)
        th, ph = oracle.init_spins(m, 0)
        ch.set_spins(th, ph)
        chs.append(ch)
        ms.append(m)
        sts.append([th, ph])
    b = g.Batch(chs)
    b.set_tuning(ppt)
    for idx in range(3):
        ro = [oracle.step(m, s[0], s[1], idx) for m, s in zip(ms, sts)]
        recs = b.step(1, force=np.array([r.accepted for r in ro]), records=True)[0]
        for r, o in zip(recs, ro):
            assert (r.site, r.u) == (o.site, o.u)
            assert abs(r.dseff - o.dseff) < FP64_DS
    b.close()


def test_zero_counts_change_nothing(g):
    # zero sweeps and zero proposals are valid calls that launch nothing
    ch, m = make(g, 4, 64, 0, seed=2)
    ch.init_spins(g.INIT_RANDOM)
    th, ph = ch.get_spins()
    mag, acc = ch.sweep(0)
    assert mag.shape == (0,) and acc == 0
    b = g.Batch([ch])
    assert b.step(0, records=True) == []
    mag, acc = b.sweep(0)
    assert mag.shape == (1, 0) and acc.tolist() == [0]
    b.close()
    th2, ph2 = ch.get_spins()
    assert np.array_equal(th, th2) and np.array_equal(ph, ph2) and ch.get_counter() == 0


@pytest.mark.parametrize("nt", [False, True])
def test_column_form_matches_one_pair_per_thread(g, nt):
    # FP32 with two site pairs per thread takes them from one y column and
    # shares the y neighbours' loads: the vectors equal those of one pair per
    # thread bit for bit (same per-site arithmetic), the block sums group the
    # sites differently.  L = 10 and 14 leave a ragged last block; 16 fills
    # its blocks.  Decisions, sites and spins equal; Delta S to rounding of the
    # FP64 sums and to the oracle.
    specs = [(10, 64, 10.0), (14, 64, 5.0), (16, 128, 20.0)]

    def run(ppt):
        chs = []
        for i, (L, M, beta) in enumerate(specs):
            ch, _ = make(g, L, M, 1, seed=51, chain_id=i, beta=beta)
            th, ph = synth.random_angles(L ** 3, 80 + i)
            ch.set_spins(th, ph)
            chs.append(ch)
        b = g.Batch(chs)
        b.set_lanes(1)
        b.set_tuning(ppt)
        b.set_nontemporal(nt)
        spins0 = [c.get_spins() for c in chs]
        recs = b.step(3, records=True)
        b.close()
        return recs, [c.get_spins() for c in chs], spins0
    r1, s1, spins0 = run(1)
    r2, s2, _ = run(2)
    for q in range(3):
        for i in range(len(specs)):
            a, c = r1[q][i], r2[q][i]
            assert (a.site, a.u, a.accepted) == (c.site, c.u, c.accepted)
            assert abs(a.dseff - c.dseff) <= 1e-11 * max(1.0, abs(a.dseff))
    for (t1, p1), (t2, p2) in zip(s1, s2):
        assert np.array_equal(t1, t2) and np.array_equal(p1, p2)
    for i, (L, M, beta) in enumerate(specs):
        m = oracle.Model(L=L, M=M, beta=beta, seed=51, chain_id=i)
        th, ph = spins0[i]
        r = r2[0][i]
        assert abs(r.dseff - oracle.delta_seff(m, th, ph, r.site, r.theta_new, r.phi_new)) < 2e-5
