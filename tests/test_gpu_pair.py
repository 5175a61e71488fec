"""GPU parity of the pair form {|o>, |v> = Delta|o>} against the oracle.

The oracle has one definition of the local moments (7 unit start vectors);
the pair form must reproduce its contracted series <o|T_n|o>, <v|T_n|v>,
<o|T_n|v> and the same Delta S_eff.  Tolerances as for the 7-vector form, with
the moments of |v> taken relative to <v|v>.
"""
import math

import numpy as np
import pytest

import oracle
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


def pair(g, L, M, prec, **kw):
    ch = g.Chain(g.Params(L=L, M=M, precision=prec, vectors=g.VECTORS_OV, **kw))
    m = oracle.Model(L=L, M=M, **{k: v for k, v in kw.items()
                                  if k in ("beta", "seed", "chain_id", "K")})
    return ch, m


@pytest.mark.parametrize("L,M", [(2, 32), (4, 256), (8, 256)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_pair_moments_match_contracted_oracle(g, L, M, prec, tol):
    if prec == 1 and L < 4:   # outside the FP32 recursion's validated range
        with pytest.raises(g.GfmcError) as e:
            pair(g, L, M, prec)
        assert e.value.status == g.GFMC_EINVAL
        return
    ch, m = pair(g, L, M, prec)
    th, ph = synth.random_angles(m.N, L + 3)
    ch.set_spins(th, ph)
    rng = np.random.default_rng(L)
    for _ in range(2):
        o = int(rng.integers(m.N))
        tn, pn = float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))
        got = ch.pair_moments(o, tn, pn)
        ref = oracle.contract(oracle.moments(m, th, ph, o), oracle.deltas(m, th, ph, o, tn, pn))
        vv0 = ref[3, 0].real
        e_oo = np.abs(got[:, 0] - ref[0]).max()
        e_vv = np.abs(got[:, 1] - ref[3]).max() / max(1.0, vv0)
        e_ov = np.abs(got[:, 2] - ref[1]).max() / max(1.0, math.sqrt(vv0))
        print(f"L={L} M={M} prec={prec} site={o}: oo {e_oo:.1e} vv {e_vv:.1e} ov {e_ov:.1e}",
              flush=True)
        assert max(e_oo, e_vv, e_ov) < tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_pair_delta_seff(g, prec, tol):
    ch, m = pair(g, 8, 512, prec, beta=20.0)
    th, ph = synth.random_angles(m.N, 5)
    ch.set_spins(th, ph)
    rng = np.random.default_rng(3)
    for _ in range(3):
        o = int(rng.integers(m.N))
        tn, pn = float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))
        got = ch.delta_seff(o, tn, pn)
        ref = oracle.delta_seff(m, th, ph, o, tn, pn)
        print(f"pair prec={prec} dS={ref:.6f} err={got - ref:.2e}", flush=True)
        assert abs(got - ref) < tol
    assert ch.delta_seff(7, th[7], ph[7]) == 0.0


def test_pair_trajectory_4cubed(g):
    ch, m = pair(g, 4, 256, 0, beta=20.0, seed=2)
    th, ph = oracle.init_spins(m, 0)
    ch.set_spins(th, ph)
    for idx in range(2 * m.N):
        ro = oracle.step(m, th, ph, idx)
        rg = ch.step(force=ro.accepted)
        assert rg.site == ro.site and rg.u == ro.u
        assert abs(rg.dseff - ro.dseff) < 1e-10
        if rg.own != ro.own:
            assert abs(math.log(ro.u) + ro.dseff) < 1e-9
    gth, gph = ch.get_spins()
    assert np.abs(gth - th).max() < 1e-13 and np.abs(gph - ph).max() < 1e-13


def test_pair_batch_alone_vs_mix(g):
    specs = [(4, 256), (6, 128), (8, 64)]

    def build():
        out = []
        for i, (L, M) in enumerate(specs):
            ch = g.Chain(g.Params(L=L, M=M, precision=1, vectors=g.VECTORS_OV, seed=9,
                                  chain_id=i, beta=10.0))
            ch.init_spins(g.INIT_RANDOM)
            out.append(ch)
        return out
    alone = [[ch.step() for _ in range(4)] for ch in build()]
    b = g.Batch(build())
    recs = b.step(4, records=True)
    b.close()
    for q in range(4):
        for i in range(len(specs)):
            r, a = recs[q][i], alone[i][q]
            assert (r.site, r.accepted, r.dseff) == (a.site, a.accepted, a.dseff)


# ------------------------------------------- the paper's mixed start vectors --
def mixed(g, L, M, prec, **kw):
    ch = g.Chain(g.Params(L=L, M=M, precision=prec, vectors=g.VECTORS_MIXED, **kw))
    m = oracle.Model(L=L, M=M, **{k: v for k, v in kw.items()
                                  if k in ("beta", "seed", "chain_id", "K", "kernel")})
    return ch, m


@pytest.mark.parametrize("L,M", [(4, 256), (8, 256)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_mixed_moments_match_literal_oracle(g, L, M, prec, tol):
    # the oracle runs four full-vector recursions on |o>, |v>, |o>+|v>, |o>+i|v>;
    # the device forms the four series from the pair recursion's sums
    ch, m = mixed(g, L, M, prec)
    th, ph = synth.random_angles(m.N, L + 11)
    ch.set_spins(th, ph)
    rng = np.random.default_rng(L + 1)
    for _ in range(2):
        o = int(rng.integers(m.N))
        tn, pn = float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))
        got = ch.mixed_moments(o, tn, pn)
        ref = oracle.mixed_moments(m, th, ph, o, tn, pn).real
        scale = np.maximum(1.0, ref[:, :1])          # moments of |v>-weighted vectors vs <a|a>
        err = (np.abs(got - ref) / scale).max(axis=1)
        print(f"mixed L={L} M={M} prec={prec} site={o}: err per vector {err}", flush=True)
        assert err.max() < tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
@pytest.mark.parametrize("kernel,K", [(0, 0), (1, 1024)])
def test_mixed_delta_seff_matches_literal_oracle(g, prec, tol, kernel, K):
    ch, m = mixed(g, 8, 512, prec, beta=20.0, kernel=kernel, K=K)
    th, ph = synth.random_angles(m.N, 6)
    ch.set_spins(th, ph)
    rng = np.random.default_rng(4)
    for _ in range(3):
        o = int(rng.integers(m.N))
        tn, pn = float(np.arccos(rng.uniform(-1, 1))), float(rng.uniform(0, 2 * np.pi))
        got = ch.delta_seff(o, tn, pn)
        ref = oracle.delta_seff_mixed(m, th, ph, o, tn, pn)
        print(f"mixed prec={prec} kernel={kernel} K={K} dS={ref:.6f} err={got - ref:.2e}",
              flush=True)
        assert abs(got - ref) < tol
    assert ch.delta_seff(7, th[7], ph[7]) == 0.0


def test_mixed_trajectory_4cubed(g):
    # teacher-forced trajectory: the mixed reconstruction drives the same chain
    ch, m = mixed(g, 4, 256, 0, beta=20.0, seed=3)
    th, ph = oracle.init_spins(m, 0)
    ch.set_spins(th, ph)
    for idx in range(m.N):
        ro = oracle.step(m, th, ph, idx)
        rg = ch.step(force=ro.accepted)
        assert rg.site == ro.site and rg.u == ro.u
        assert abs(rg.dseff - ro.dseff) < 1e-10
    gth, gph = ch.get_spins()
    assert np.abs(gth - th).max() < 1e-13 and np.abs(gph - ph).max() < 1e-13


def test_mixed_and_pair_chains_in_one_batch(g):
    # both forms share the pair recursion (one launch per step for the batch)
    # and differ only in the reconstruction; each equals its alone run
    specs = [(4, 256, 1), (6, 128, 2), (8, 64, 2), (4, 64, 1)]

    def build():
        out = []
        for i, (L, M, vec) in enumerate(specs):
            ch = g.Chain(g.Params(L=L, M=M, precision=1, vectors=vec, seed=12, chain_id=i,
                                  beta=10.0))
            ch.init_spins(g.INIT_RANDOM)
            out.append(ch)
        return out
    alone = [[ch.step() for _ in range(3)] for ch in build()]
    b = g.Batch(build())
    recs = b.step(3, records=True)
    b.close()
    for q in range(3):
        for i in range(len(specs)):
            r, a = recs[q][i], alone[i][q]
            assert (r.site, r.accepted, r.dseff) == (a.site, a.accepted, a.dseff)


# --------------------------------------------- two steps per launch (shape 3) --
# (L, M, K): S = M/2 of 64, 45, 32 and 31 steps, so the chains drop out of the
# two-step launches at different points, two of them with a last step alone
TWO_STEP_SPECS = [(16, 128, 128), (8, 90, 128), (24, 64, 64), (16, 62, 64)]


def _two_step_batch(g, prec, shape, vectors):
    chs = []
    for i, (L, M, K) in enumerate(TWO_STEP_SPECS):
        ch = g.Chain(g.Params(L=L, M=M, K=K, precision=prec, vectors=vectors, seed=21,
                              chain_id=i, beta=10.0))
        th, ph = synth.random_angles(L ** 3, 40 + i)
        ch.set_spins(th, ph)
        chs.append(ch)
    b = g.Batch(chs)
    b.set_lanes(1)
    b.set_tuning(shape)
    assert b.tuning() == (shape, 1)
    return chs, b


@pytest.mark.parametrize("prec,vectors", [(0, 1), (1, 1), (1, 2)])
def test_two_step_shape_matches_one_step_shape_and_oracle(g, prec, vectors):
    # Shapes 2 (two site pairs of a y column per thread, sharing their y
    # neighbours' loads) and 3 (two steps per launch) form the same vector
    # values as shape 1 (same arithmetic, term for term) and sum them in
    # another order: every proposal's Delta S agrees to rounding of the FP64
    # sums, the decisions and final spins are equal, and the first proposal's
    # Delta S matches the oracle.  L = 24 puts row ends inside blocks.
    nprop = 3
    runs = {}
    for shape in (1, 2, 3):
        chs, b = _two_step_batch(g, prec, shape, vectors)
        spins0 = [c.get_spins() for c in chs]
        recs = b.step(nprop, records=True)
        b.close()
        runs[shape] = (recs, [c.get_spins() for c in chs], spins0)
    r1, s1, spins0 = runs[1]
    tol = 1e-10 if prec == 0 else 2e-5
    for shape in (2, 3):
        r3, s3, _ = runs[shape]
        for q in range(nprop):
            for i in range(len(TWO_STEP_SPECS)):
                a, b_ = r1[q][i], r3[q][i]
                print(f"shape {shape} prop {q} chain {i}: dS {a.dseff:.12f} / {b_.dseff:.12f}",
                      flush=True)
                assert (a.site == b_.site and a.theta_new == b_.theta_new
                        and a.phi_new == b_.phi_new)
                assert abs(a.dseff - b_.dseff) < 1e-9 * max(1.0, abs(a.dseff))
                assert a.accepted == b_.accepted
        for (t1, p1), (t3, p3) in zip(s1, s3):
            assert np.array_equal(t1, t3) and np.array_equal(p1, p3)
        for i, (L, M, K) in enumerate(TWO_STEP_SPECS):
            m = oracle.Model(L=L, M=M, K=K, beta=10.0, seed=21, chain_id=i)
            th, ph = spins0[i]
            r = r3[0][i]
            ref = (oracle.delta_seff(m, th, ph, r.site, r.theta_new, r.phi_new) if vectors == 1
                   else oracle.delta_seff_mixed(m, th, ph, r.site, r.theta_new, r.phi_new))
            print(f"shape {shape} chain {i} L={L} M={M}: dS {r.dseff:.10f} oracle {ref:.10f}",
                  flush=True)
            assert abs(r.dseff - ref) < tol


def test_two_step_shape_refusals(g):
    def batch(L, M, vectors, prec=0):
        ch = g.Chain(g.Params(L=L, M=M, precision=prec, vectors=vectors, seed=3))
        return g.Batch([ch, g.Chain(g.Params(L=L, M=M, precision=prec, vectors=vectors,
                                             seed=4))])
    for L, vec in ((16, 0), (12, 1), (6, 1)):   # 7-vector form; too few blocks; L < 8
        b = batch(L, 64, vec)
        with pytest.raises(g.GfmcError) as e:
            b.set_tuning(3)
        assert e.value.status == g.GFMC_EINVAL
        b.close()
    b = batch(16, 64, 1)
    b.set_tuning(3)
    with pytest.raises(g.GfmcError) as e:
        b.set_schedule(True)           # the two-step shape is lock-step only
    assert e.value.status == g.GFMC_EINVAL
    b.set_tuning(1)
    b.set_schedule(True)
    with pytest.raises(g.GfmcError) as e:
        b.set_tuning(3)
    assert e.value.status == g.GFMC_EINVAL
    b.close()
