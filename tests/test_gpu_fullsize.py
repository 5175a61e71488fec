"""Full-size GPU checks: the 64^3 (M = 4096) and 32^3 (M = 2048) shapes.

At 64^3 the oracle needs minutes per site, so the checks use what holds at any
size: for uniform spins H is the tight-binding operator and its local moments
are the exact k-sums (1/N) sum_q cos(q.(r_j - r_k)) T_n(e_q / a); for random
spins the moment invariants (mu_0, mu_1, mu_2^{oo}, Hermiticity, bipartite
zeros, |mu| <= 1).  At 32^3 the oracle is run one site / one proposal at a time.
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


def ksum_classes(L, M, a):
    """Exact moments of the uniform-spin lattice for displacement classes
    0, e_x, 2 e_x, e_x + e_y (cubic symmetry makes every pair of the 7 start
    sites fall in one of them); Chebyshev recursion on the q grid."""
    q1 = 2 * np.pi * np.arange(L) / L
    c = np.cos(q1)
    x = ((-2.0 / a) * (c[:, None, None] + c[None, :, None] + c[None, None, :])).ravel()
    disps = [(0, 0, 0), (1, 0, 0), (2, 0, 0), (1, 1, 0)]
    ph = np.stack([np.cos(q1[:, None, None] * D[0] + q1[None, :, None] * D[1] +
                          q1[None, None, :] * D[2]).ravel() for D in disps])
    out = np.zeros((M, 4))
    t0, t1 = np.ones_like(x), x.copy()
    out[0], out[1] = ph @ t0 / x.size, ph @ t1 / x.size
    for n in range(2, M):
        t0, t1 = t1, 2 * x * t1 - t0
        out[n] = ph @ t1 / x.size
    return out


def class_of(L, i, j):
    ri = np.array([i % L, (i // L) % L, i // (L * L)])
    rj = np.array([j % L, (j // L) % L, j // (L * L)])
    d = np.abs(ri - rj)
    d = np.minimum(d, L - d)
    key = tuple(sorted(d.tolist(), reverse=True))
    return {(0, 0, 0): 0, (1, 0, 0): 1, (2, 0, 0): 2, (1, 1, 0): 3}[key]


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_64cubed_uniform_spins_k_sum(g, prec, tol):
    L, M = 64, 4096
    ch = g.Chain(g.Params(L=L, M=M, precision=prec))
    ch.init_spins(g.INIT_FM)
    o = 123457
    mu = ch.moments(o)
    a = 6.0 / 0.99
    ref_c = ksum_classes(L, M, a)
    s = oracle.start_sites(L, o)
    ref = np.zeros((M, 7, 7))
    for j in range(7):
        for k in range(7):
            ref[:, j, k] = ref_c[:, class_of(L, s[j], s[k])]
    err = np.abs(mu - ref).max()
    print(f"64^3 M=4096 prec={prec} uniform spins: max|dmu|={err:.2e}", flush=True)
    assert err < tol


def test_64cubed_random_spins_invariants(g):
    L, M = 64, 4096
    ch64 = g.Chain(g.Params(L=L, M=M, precision=0, seed=11))
    ch64.init_spins(g.INIT_RANDOM)
    th, ph = ch64.get_spins()
    o = 200001
    mu = ch64.moments(o)
    s = oracle.start_sites(L, o)
    a = 6.0 / 0.99
    # mu_1 = Ht between start sites, from the angles (equation "ht")
    H1 = np.zeros((7, 7), complex)
    for j in range(7):
        for k in range(7):
            for d in range(6):
                if oracle.neighbor(L, s[j], d) == s[k]:
                    H1[j, k] += -oracle.hopping(th[s[j]], ph[s[j]], th[s[k]], ph[s[k]]) / a
    assert np.abs(mu[0] - np.eye(7)).max() == 0
    assert np.abs(mu[1] - H1).max() < 1e-15
    S = lambda t, p: np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
    t2 = sum((1 + S(th[o], ph[o]) @ S(th[n], ph[n])) / 2 for n in s[1:])
    assert abs(mu[2, 0, 0] - (2 * t2 / a ** 2 - 1)) < 1e-14
    assert np.abs(mu - mu.conj().transpose(0, 2, 1)).max() == 0
    assert np.abs(mu).max() <= 1 + 1e-12
    assert np.all(mu[1::2, 0, 0] == 0) and np.all(mu[0::2, 0, 1:] == 0)
    assert np.all(mu[1::2, 1:, 1:] == 0)
    # FP32 recursion on the same spins stays within the FP32 tolerance
    ch32 = g.Chain(g.Params(L=L, M=M, precision=1, seed=11))
    ch32.set_spins(th, ph)
    err = np.abs(ch32.moments(o) - mu).max()
    print(f"64^3 random spins: FP32 vs FP64 max|dmu|={err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_32cubed_delta_seff_against_oracle(g, prec, tol):
    L, M = 32, 2048
    ch = g.Chain(g.Params(L=L, M=M, beta=1 / 0.05, precision=prec, seed=7, chain_id=1))
    m = oracle.Model(L=L, M=M, beta=1 / 0.05, seed=7, chain_id=1)
    th, ph = oracle.init_spins(m, 0)
    ch.set_spins(th, ph)
    for idx in range(2):
        ro = oracle.step(m, th, ph, idx)
        rg = ch.step(force=ro.accepted)
        print(f"32^3 prec={prec} proposal {idx}: dS={ro.dseff:.9f} err={rg.dseff - ro.dseff:.2e}",
              flush=True)
        assert rg.site == ro.site and rg.u == ro.u
        assert abs(rg.dseff - ro.dseff) < tol


def test_64cubed_with_eight_32cubed_chains_in_one_batch(g):
    # one 64^3 chain (M = 4096) and eight 32^3 chains (M = 2048), FP32
    # recursion: each chain's proposal in the mixed batch equals its alone run
    def build():
        chs = [g.Chain(g.Params(L=64, M=4096, beta=20.0, precision=1, seed=11, chain_id=0))]
        for c in range(8):
            chs.append(g.Chain(g.Params(L=32, M=2048, beta=20.0, precision=1, seed=11,
                                        chain_id=1 + c)))
        for ch in chs:
            ch.init_spins(g.INIT_RANDOM)
        return chs
    alone = [ch.step() for ch in build()]
    mixed = build()
    b = g.Batch(mixed)
    recs = b.step(1, records=True)[0]
    b.close()
    for r, a in zip(recs, alone):
        assert (r.site, r.u, r.accepted) == (a.site, a.u, a.accepted)
        assert r.dseff == a.dseff


@pytest.mark.parametrize("tuning", [(1, 2, 512), (2, 2, 256)])
def test_mixed_benchmark_batch_against_oracle(g, tuning):
    # The mixed benchmark's workload: one 64^3 chain (M = 4096, chain_id 0)
    # and eight 32^3 chains (M = 2048, chain_id 1..8), FP32 recursion,
    # beta = 20, seed 11, uniform-sphere starts drawn on the device, in the
    # launch shapes its autotuner picks (one site pair per thread in
    # 512-thread blocks, or two pairs of a y column; two lanes).
    # A lock-step proposal with forced decisions: the 64^3 chain's against the
    # oracle's stored first proposal, two 32^3 chains against the oracle.
    # Then one step-granular window (2048 rounds) from there: the 32^3 chains
    # make two proposals, the 64^3 chain one, and each chain ends where it
    # ends alone (a batch of its own with the same launch shape): spins bit
    # for bit.
    import json
    import os
    ppt, lanes, bt = tuning
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_dseff_64cubed.json")
    gold = json.load(open(path))["proposals"][0]
    specs = [(64, 4096, 0)] + [(32, 2048, 1 + c) for c in range(8)]

    def chain(L, M, cid):
        ch = g.Chain(g.Params(L=L, M=M, beta=20.0, precision=1, seed=11, chain_id=cid))
        ch.init_spins(g.INIT_RANDOM)
        return ch

    def shape(b, nl):
        b.set_tuning(ppt)
        b.set_lanes(nl)
        b.set_block_threads(bt)

    sample = [2, 7]
    force = np.full(len(specs), -1, dtype=np.int32)
    force[0] = gold["accepted"]
    ref = {}
    for i in sample:
        L, M, cid = specs[i]
        m = oracle.Model(L=L, M=M, beta=20.0, seed=11, chain_id=cid)
        th, ph = oracle.init_spins(m, 0)
        ref[i] = oracle.step(m, th, ph, 0)
        force[i] = ref[i].accepted
    chs = [chain(*s) for s in specs]
    b = g.Batch(chs)
    shape(b, lanes)
    recs = b.step(1, force=force, records=True)[0]
    r = recs[0]
    print(f"mixed shape={tuning} 64^3: dS={gold['dseff']:.9f} err={r.dseff - gold['dseff']:.2e}",
          flush=True)
    assert (r.index, r.site, r.u, r.accepted) == (gold["index"], gold["site"], gold["u"],
                                                  gold["accepted"])
    assert abs(r.dseff - gold["dseff"]) < 2e-5
    for i in sample:
        a, o = recs[i], ref[i]
        print(f"mixed shape={tuning} 32^3 chain {i}: dS={o.dseff:.9f} err={a.dseff - o.dseff:.2e}",
              flush=True)
        assert (a.site, a.u, a.accepted) == (o.site, o.u, o.accepted)
        assert abs(a.dseff - o.dseff) < 2e-5
    b.set_schedule(True)
    b.step(1)
    counters = [c.get_counter() for c in chs]
    assert counters == [2] + [3] * 8
    got = [c.get_spins() for c in chs]
    b.close()
    for i, (L, M, cid) in enumerate(specs):
        ch = chain(L, M, cid)
        bb = g.Batch([ch])
        shape(bb, 1)
        assert bb.form()["persistent"] == 0 and bb.form()["resident"] == 0
        bb.step(1, force=force[i:i + 1])
        bb.step(counters[i] - 1)
        bb.close()
        th, ph = ch.get_spins()
        assert ch.get_counter() == counters[i]
        assert np.array_equal(th, got[i][0]) and np.array_equal(ph, got[i][1])


@pytest.mark.parametrize("vectors,tuning", [(0, None), (0, (2, 2, 256)), (0, (1, 2, 512)),
                                            (1, None)])
def test_benchmark_batch_sampled_against_oracle(g, vectors, tuning):
    # The benchmark's workload: 64 chains of 32^3, M = 2048, FP32 recursion,
    # T = 0.02..0.2 t, uniform-sphere starts drawn on the device (seed 7,
    # chain_id = chain index), with the autotuned launch shape and with the
    # two shapes the benchmark's autotuner picks for it (two site pairs of a
    # y column per thread, or one with 512-thread blocks; two lanes).  One
    # batched proposal; sampled chains are checked against the oracle one
    # proposal at a time, the decisions of the sampled chains taken from the
    # oracle.
    import synth
    L, M, n = 32, 2048, 64
    temps = synth.temperature_ladder(n, 0.02, 0.2)
    chs = [g.Chain(g.Params(L=L, M=M, beta=1.0 / temps[c], precision=1, seed=7, chain_id=c,
                            vectors=vectors))
           for c in range(n)]
    for ch in chs:
        ch.init_spins(g.INIT_RANDOM)
    b = g.Batch(chs)
    if tuning is None:
        ppt = b.autotune(16)
    else:
        ppt, lanes, bt = tuning
        b.set_lanes(lanes)
        b.set_block_threads(bt)
        b.set_tuning(ppt)
    sample = [0, 37, 63] if vectors == 0 else [11, 50]
    force = np.full(n, -1, dtype=np.int32)
    ref = {}
    for c in sample:
        m = oracle.Model(L=L, M=M, beta=1.0 / temps[c], seed=7, chain_id=c)
        th, ph = oracle.init_spins(m, 0)
        ref[c] = oracle.step(m, th, ph, 0)
        force[c] = ref[c].accepted
    recs = b.step(1, force=force, records=True)[0]
    b.close()
    for c in sample:
        r, o = recs[c], ref[c]
        print(f"bench batch vectors={vectors} shape={ppt} chain {c}: dS={o.dseff:.8f} "
              f"err={r.dseff - o.dseff:.2e}", flush=True)
        assert r.site == o.site and r.u == o.u and r.accepted == o.accepted
        assert abs(r.dseff - o.dseff) < 2e-5


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_64cubed_delta_seff_against_stored_oracle(g, prec, tol):
    # The oracle's first two proposals of a 64^3, M = 4096 chain (beta = 20,
    # seed 11), stored by tests/golden/make_golden.py: the oracle needs
    # minutes per proposal at this size.  Same starts (the oracle's own
    # initial spins), decisions forced to the oracle's.
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_dseff_64cubed.json")
    ref = json.load(open(path))
    m = oracle.Model(L=64, M=4096, beta=20.0, seed=11, chain_id=0)
    th, ph = oracle.init_spins(m, 0)
    ch = g.Chain(g.Params(L=64, M=4096, beta=20.0, precision=prec, seed=11, chain_id=0))
    ch.set_spins(th, ph)
    for rp in ref["proposals"]:
        r = ch.step(force=rp["accepted"])
        print(f"64^3 prec={prec} proposal {rp['index']}: dS={rp['dseff']:.9f} "
              f"err={r.dseff - rp['dseff']:.2e}", flush=True)
        assert (r.index, r.site, r.u) == (rp["index"], rp["site"], rp["u"])
        assert abs(r.theta_new - rp["theta_new"]) <= 4 * np.spacing(max(rp["theta_new"], 1.0))
        assert abs(r.dseff - rp["dseff"]) < tol


def test_largest_lattice_256cubed_against_oracle(g):
    # L = 256 is the largest lattice the library accepts (N = 2^24 sites,
    # 32768 blocks of the step kernel): moments at the last site (every
    # neighbour wraps around) against the oracle in both precisions, and the
    # closed forms of mu_0, mu_1, mu_2^{oo} at sites across the lattice
    L, M = 256, 4
    m = oracle.Model(L=L, M=M, seed=0)
    th, ph = synth.random_angles(m.N, 296)
    o = m.N - 1
    ref = oracle.moments(m, th, ph, o)
    a = 6.0 / 0.99
    S = lambda t, p: np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        ch = g.Chain(g.Params(L=L, M=M, precision=prec, seed=0))
        ch.set_spins(th, ph)
        err = np.abs(ch.moments(o) - ref).max()
        print(f"256^3 M=4 prec={prec} site {o}: max|dmu|={err:.2e}", flush=True)
        assert err < tol
        for x in (0, 1 << 23, 12345677, m.N - L * L):
            mu = ch.moments(x)
            s = oracle.start_sites(L, x)
            assert np.abs(mu[0] - np.eye(7)).max() == 0
            h = [-oracle.hopping(th[x], ph[x], th[n], ph[n]) / a for n in s[1:]]
            assert np.abs(mu[1, 0, 1:] - h).max() < (1e-15 if prec == 0 else 1e-7)
            t2 = sum((1 + S(th[x], ph[x]) @ S(th[n], ph[n])) / 2 for n in s[1:])
            assert abs(mu[2, 0, 0] - (2 * t2 / a ** 2 - 1)) < (1e-14 if prec == 0 else 1e-6)
        ch.close()
