"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test compares the oracle with something other than itself: numpy's own
Philox, exact diagonalisation of a Hamiltonian built from a different formula,
closed forms (tight-binding band, geometric series, Fermi integral, high-T
expansion), exact invariants, or brute-force constructions.  None of these
needs a GPU.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import ed


# ------------------------------------------------------------------ RNG ----
@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 1, 0, 0), (42, 7)),
                                     ((2**64 - 1, 3, 0, 0), (1, 2)),
                                     ((123456789, 2, 0, 0), (2**63 + 5, 2**40))])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox(4x64-10) increments its 256-bit counter before each block.
    c = ctr[0] + (ctr[1] << 64) + (ctr[2] << 128) + (ctr[3] << 192)
    g = np.random.Philox(counter=(c - 1) % 2**256, key=key[0] + (key[1] << 64))
    assert oracle.philox(ctr, key) == [int(g.random_raw()) for _ in range(4)]


def test_index_and_uniform_maps():
    rng = np.random.default_rng(0)
    for r in [0, 1, 2**64 - 1, 2**63] + [int(x) for x in rng.integers(0, 2**63, 20)]:
        for n in [8, 64, 4096, 32768, 262144, 12345]:
            assert oracle.mulhi_index(r, n) == (r * n) >> 64
        assert oracle.u01(r) == (r >> 11) / 2.0**53
    assert oracle.u01(2**64 - 1) < 1.0


# -------------------------------------------------------------- model ----
def test_hopping_spinor_identity_and_modulus():
    th, ph = synth.random_angles(200, 11)
    chi = ed.spinor(th, ph)
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    for i in range(0, 200, 2):
        j = i + 1
        t = oracle.hopping(th[i], ph[i], th[j], ph[j])
        assert abs(t - np.vdot(chi[i], chi[j])) < 1e-15
        assert abs(abs(t) ** 2 - (1 + S[i] @ S[j]) / 2) < 1e-15
        assert abs(oracle.hopping(th[j], ph[j], th[i], ph[i]) - np.conj(t)) < 1e-16


@pytest.mark.parametrize("L", [2, 3, 4])
def test_dense_hamiltonian_structure(L):
    m = oracle.Model(L=L)
    th, ph = synth.random_angles(m.N, L)
    Ht = oracle.dense_ht(m, th, ph)
    H = ed.hamiltonian(L, th, ph)
    assert np.abs(Ht - H / m.scale_a()).max() < 1e-15
    assert np.abs(Ht - Ht.conj().T).max() == 0.0
    e = np.linalg.eigvalsh(H)
    assert e.min() >= -6.0 - 1e-12 and e.max() <= 6.0 + 1e-12   # Gershgorin, |t_ij| <= 1
    if L % 2 == 0:   # bipartite lattice: spectrum symmetric about 0
        assert np.abs(np.sort(e) - np.sort(-e)).max() < 1e-12


@pytest.mark.parametrize("L", [3, 4])
def test_ferromagnet_is_tight_binding(L):
    th, ph = synth.ferro_angles(L ** 3, 0.7, 1.9)
    e = np.sort(np.linalg.eigvalsh(oracle.dense_ht(oracle.Model(L=L, a=1.0), th, ph)))
    q = 2 * np.pi * np.arange(L) / L
    ek = -2 * (np.cos(q)[:, None, None] + np.cos(q)[None, :, None] + np.cos(q)[None, None, :])
    assert np.abs(e - np.sort(ek.ravel())).max() < 1e-12


# ------------------------------------------------------------ moments ----
@pytest.mark.parametrize("L,M,seed,o", [(2, 64, 1, 3), (3, 96, 2, 13), (4, 128, 3, 37),
                                        (4, 128, 4, 0)])
def test_moments_match_exact_diagonalisation(L, M, seed, o):
    m = oracle.Model(L=L, M=M)
    th, ph = synth.random_angles(m.N, seed)
    mu = oracle.moments(m, th, ph, o)
    s = oracle.start_sites(L, o)
    assert s == [o] + [ed.nbr(L, o, d) for d in range(6)]
    ref = ed.cheb_moments_ed(ed.hamiltonian(L, th, ph) / m.scale_a(), s, s, M)
    assert np.abs(mu - ref).max() < 1e-12


@pytest.mark.parametrize("L,M", [(6, 256), (8, 128)])
def test_moments_ferromagnet_k_sum(L, M):
    # Uniform spins: t_ij = 1, and <j|T_n(Ht)|k> = (1/N) sum_q e^{iq(r_j - r_k)} T_n(e_q / a).
    m = oracle.Model(L=L, M=M)
    th, ph = synth.ferro_angles(m.N, 1.2, 0.3)
    o = 17
    mu = oracle.moments(m, th, ph, o)
    s = oracle.start_sites(L, o)
    r = np.array([[i % L, (i // L) % L, i // (L * L)] for i in s])
    q1 = 2 * np.pi * np.arange(L) / L
    Q = np.stack(np.meshgrid(q1, q1, q1, indexing='ij'), -1).reshape(-1, 3)
    eq = -2 * np.cos(Q).sum(1) / m.scale_a()
    # global U(1) gauge of the uniform spinor: t_ij = 1 exactly only if phases match
    chi = ed.spinor(th[:1], ph[:1])[0]
    assert abs(np.vdot(chi, chi) - 1) < 1e-15
    T = np.cos(np.arange(M)[:, None] * np.arccos(eq)[None, :])
    phase = np.exp(1j * np.einsum('qa,jka->qjk', Q, r[:, None, :] - r[None, :, :]))
    ref = np.einsum('nq,qjk->njk', T, phase) / m.N
    assert np.abs(mu - ref).max() < 1e-12


def test_moment_invariants():
    L, M = 4, 200
    m = oracle.Model(L=L, M=M)
    th, ph = synth.random_angles(m.N, 9)
    o = 22
    mu = oracle.moments(m, th, ph, o)
    s = oracle.start_sites(L, o)
    Ht = oracle.dense_ht(m, th, ph)
    assert np.abs(mu[0] - np.eye(7)).max() == 0.0
    assert np.abs(mu[1] - Ht[np.ix_(s, s)]).max() < 1e-16
    assert np.abs(mu).max() <= 1.0 + 1e-12
    assert np.abs(mu - mu.conj().transpose(0, 2, 1)).max() < 1e-13
    # bipartite: <j|Ht^n|k> = 0 unless n = dist(j,k) mod 2 -> o-o odd, o-n even, n-n odd vanish
    assert np.all(mu[1::2, 0, 0] == 0) and np.all(mu[0::2, 0, 1:] == 0)
    assert np.all(mu[1::2, 1:, 1:] == 0)
    # mu_2^{oo} = 2 <o|Ht^2|o> - 1 = 2 (t/a)^2 sum_d |t_{o n_d}|^2 - 1
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    t2 = sum((1 + S[o] @ S[n]) / 2 for n in s[1:])
    assert abs(mu[2, 0, 0] - (2 * t2 / m.scale_a() ** 2 - 1)) < 1e-15


def test_l2_doubled_bonds_and_coinciding_sites():
    m = oracle.Model(L=2, M=32)
    th, ph = synth.random_angles(8, 5)
    s = oracle.start_sites(2, 6)
    assert s[1] == s[2] and s[3] == s[4] and s[5] == s[6]
    mu = oracle.moments(m, th, ph, 6)
    assert mu[0, 1, 2] == 1.0
    ref = ed.cheb_moments_ed(ed.hamiltonian(2, th, ph) / m.scale_a(), s, s, 32)
    assert np.abs(mu - ref).max() < 1e-13


# -------------------------------------------------------- contraction ----
def test_contraction_matches_vector_v():
    L, M = 4, 96
    m = oracle.Model(L=L, M=M)
    th, ph = synth.random_angles(m.N, 21)
    o, tn, pn = 9, 2.0, 0.5
    dl = oracle.deltas(m, th, ph, o, tn, pn)
    # Delta = H' - H from two full Hamiltonians
    th2, ph2 = th.copy(), ph.copy()
    th2[o], ph2[o] = tn, pn
    D = ed.hamiltonian(L, th2, ph2) - ed.hamiltonian(L, th, ph)
    s = oracle.start_sites(L, o)
    assert np.abs(np.array([D[n, o] for n in s[1:]]) - dl).max() < 1e-15
    assert abs(D[o, o]) < 1e-15
    v = D[:, o]                                       # |v> = Delta |o>
    e, U = np.linalg.eigh(ed.hamiltonian(L, th, ph) / m.scale_a())
    T = np.cos(np.arange(M)[:, None] * np.arccos(np.clip(e, -1, 1))[None, :])
    Uo, Uv = U[o, :], v.conj() @ U                    # <o|l>, <v|l>
    ref = {"oo": T @ (Uo * Uo.conj()), "ov": T @ (Uo * Uv.conj()),
           "vo": T @ (Uv * Uo.conj()), "vv": T @ (Uv * Uv.conj())}
    got = oracle.contract(oracle.moments(m, th, ph, o), dl)
    for i, k in enumerate(["oo", "ov", "vo", "vv"]):
        assert np.abs(got[i] - ref[k]).max() < 1e-12, k


# --------------------------------------------------------- transform ----
def test_jackson_and_lorentz_coefficients():
    M = 64
    g = oracle.kernel_coeffs(M, 0)
    assert abs(g[0] - 1.0) < 1e-15 and np.all(np.diff(g) < 0) and g[-1] > 0
    # Jackson damping of a single level is a positive kernel: sum_n (2-d_n0) g_n cos(n x) >= 0
    x = np.linspace(0, np.pi, 501)
    ker = g[0] + 2 * (g[1:, None] * np.cos(np.arange(1, M)[:, None] * x[None, :])).sum(0)
    assert ker.min() > -1e-12


@pytest.mark.parametrize("M,lam", [(64, 4.0), (256, 4.0), (100, 1.5), (2048, 6.0)])
def test_lorentz_coefficients_solve_their_boundary_value_problem(M, lam):
    # The Lorentz damping factors are the unique solution of the second-order
    # linear recurrence g_{n+1} + g_{n-1} = 2 cosh(lambda/M) g_n with g_0 = 1
    # and g_M = 0 (a decaying exponential pushed to zero at n = M; the KPM
    # review cited by the paper derives the kernel this way).  The check never
    # evaluates the closed form: it tests the recurrence, both boundary values
    # (g_M from extending the recurrence one step past n = M - 1), and that g
    # falls monotonically from 1 towards 0.
    g = oracle.kernel_coeffs(M, 1, lam)
    c = 2.0 * math.cosh(lam / M)
    assert g.shape == (M,) and g[0] == 1.0
    res = g[2:] + g[:-2] - c * g[1:-1]
    assert np.abs(res).max() < 1e-13
    g_M = c * g[M - 1] - g[M - 2]
    assert abs(g_M) < 1e-13
    assert np.all(np.diff(g) < 0) and g[-1] > 0
    # damping close to e^{-lambda n / M} away from n = M: a Lorentzian of width lambda / M
    n = np.arange(M // 2)
    assert np.abs(g[: M // 2] / np.exp(-lam * n / M) - 1).max() < 2 * math.exp(-lam)


@pytest.mark.parametrize("M,K,alpha", [(64, 64, 0.7), (128, 256, 2.1), (50, 64, 1.3)])
def test_green_direct_sum_closed_form(M, K, alpha):
    # One level at cos(alpha), no damping: mu_n = cos(n alpha); the sum of
    # mu'_n e^{-i n th} is a pair of geometric series.
    mu = np.cos(np.arange(M) * alpha).astype(complex)
    G = oracle.green(mu, np.ones(M), K)
    th = np.pi * (np.arange(K) + 0.5) / K

    def geo(x):   # sum_{n=1}^{M-1} e^{i n x}
        return np.exp(1j * x) * (1 - np.exp(1j * (M - 1) * x)) / (1 - np.exp(1j * x))
    s = 0.5 + 0.5 * (geo(alpha - th) + geo(-alpha - th))
    ref = 2j * s / np.sin(th)
    assert np.abs(G - ref).max() < 1e-10 * np.abs(ref).max()


def test_green_roundtrip_discrete_orthogonality():
    # (1/K) sum_k T_n(w_k) sin(th_k) Im Gt(w_k) = g_n mu_n for real moments, n < K.
    L, M = 4, 128
    m = oracle.Model(L=L, M=M)
    th, ph = synth.random_angles(m.N, 4)
    mu = oracle.moments(m, th, ph, 5)[:, 0, 0]
    g = oracle.kernel_coeffs(M)
    for K in (M, 2 * M):
        G = oracle.green(mu, g, K)
        thk = np.pi * (np.arange(K) + 0.5) / K
        back = (np.cos(np.arange(M)[:, None] * thk[None, :]) * np.sin(thk) * G.imag).sum(1) / K
        assert np.abs(back - g * mu.real).max() < 1e-13
    assert abs(back[0] - 1.0) < 1e-13      # sum rule: mu_0 = g_0 = 1


def test_green_converges_to_resolvent_off_the_band():
    # At nodes more than 0.1 away from every level the damped series approaches
    # the resolvent <o|(Ht - w)^-1|o> (real) and its imaginary part vanishes,
    # with an error shrinking roughly as M^-2 (fixes sign and scale of Re G).
    L = 4
    m = oracle.Model(L=L)
    th, ph = synth.ferro_angles(m.N)
    e, U = np.linalg.eigh(oracle.dense_ht(m, th, ph))
    wt = np.abs(U[0, :]) ** 2
    lev = np.unique(np.round(e[wt > 1e-12], 12))
    errs = []
    for M in (1024, 2048):
        m.M = M
        mu = oracle.moments(m, th, ph, 0)[:, 0, 0]
        G = oracle.green(mu, oracle.kernel_coeffs(M), M)
        w = np.cos(np.pi * (np.arange(M) + 0.5) / M)
        far = np.min(np.abs(w[:, None] - lev[None, :]), 1) > 0.1
        ref = (wt[None, :] / (e[None, :] - w[:, None])).sum(1)
        assert far.sum() > M // 4
        errs.append(max(np.abs(G.real[far] - ref[far]).max(), np.abs(G.imag[far]).max()))
    assert errs[1] < 1e-3 and errs[0] / errs[1] > 3.0


# ---------------------------------------------------- determinant ----
def test_determinant_formula_with_exact_resolvent():
    L = 4
    m = oracle.Model(L=L)
    a = m.scale_a()
    th, ph = synth.random_angles(m.N, 8)
    o, tn, pn = 30, 0.3, 4.0
    th2, ph2 = th.copy(), ph.copy()
    th2[o], ph2[o] = tn, pn
    H, H2 = ed.hamiltonian(L, th, ph), ed.hamiltonian(L, th2, ph2)
    D = H2 - H
    v = D[:, o]
    e, e2 = np.linalg.eigvalsh(H), np.linalg.eigvalsh(H2)
    for z in [0.3 + 0.2j, -2.1 + 0.05j, 1.7 + 1.0j]:
        R = np.linalg.inv(H / a - (z / a) * np.eye(m.N))      # rescaled resolvent
        Gt = {"oo": R[o, o], "ov": R[o, :] @ v, "vo": v.conj() @ R[:, o],
              "vv": v.conj() @ R @ v}
        d = oracle.det(a, *[np.array([Gt[k]]) for k in ["oo", "ov", "vo", "vv"]])[0]
        full = np.linalg.det(np.eye(m.N) + np.linalg.inv(H - z * np.eye(m.N)) @ D)
        prod = np.prod((e2 - z) / (e - z))
        assert abs(d - full) < 1e-12 * abs(full) and abs(d - prod) < 1e-11 * abs(prod)


# ----------------------------------------------------------- phase ----
def test_phase_scan_unwraps_from_the_lowest_node():
    K = 400
    k = np.arange(K)
    psi = 2.9 * np.pi * np.sin(np.pi * (K - 1 - k) / (K - 1)) ** 2 + 0.3 * (K - 1 - k) / K
    psi[-1] = 0.0
    d = (1.0 + 0.5 * np.cos(k)) * np.exp(1j * psi)
    phi = oracle.phase(d)
    assert np.abs(phi - psi).max() < 1e-12
    # anchored by the principal argument at the lowest node
    d2 = d * np.exp(1j * 0.4)
    assert np.abs(oracle.phase(d2) - (psi + 0.4)).max() < 1e-12


# ------------------------------------------------------ quadrature ----
@pytest.mark.parametrize("beta,mu", [(1.0, 0.0), (3.0, 0.7), (0.2, -1.0)])
def test_quadrature_of_constant_phase_is_fermi_integral(beta, mu):
    # Midpoint rule in theta: the integrand F(cos th) |sin th| has kinks at
    # 0 and pi, so the error is c/K^2 with a fixed c; check the order and size.
    a, b, c = 6.0 / 0.99, 0.0, 0.37
    F = lambda E: E - np.logaddexp(0.0, beta * (E - mu)) / beta    # antiderivative of f
    ref = beta / np.pi * c * (F(a + b) - F(-a + b))
    err = [oracle.quadrature(K, beta, mu, a, b, np.full(K, c)) - ref for K in (256, 512, 1024)]
    assert abs(err[2]) < 1e-5 * max(1.0, abs(ref))
    assert abs(err[0] / err[1] - 4.0) < 0.05 and abs(err[1] / err[2] - 4.0) < 0.05


# --------------------------------------------------------- Delta S ----
def test_identity_proposal_gives_zero():
    m = oracle.Model(L=4, M=128)
    th, ph = synth.random_angles(m.N, 3)
    assert oracle.delta_seff(m, th, ph, 12, th[12], ph[12]) == 0.0


def test_gauge_invariance():
    m = oracle.Model(L=4, M=128, beta=5.0)
    th, ph = synth.random_angles(m.N, 31)
    o, tn, pn = 40, 1.0, 3.0
    ds = oracle.delta_seff(m, th, ph, o, tn, pn)
    # a uniform shift of every azimuth is a diagonal unitary on H
    ds2 = oracle.delta_seff(m, th, ph + 0.77, o, tn, pn + 0.77)
    assert abs(ds - ds2) < 1e-11
    # a global rotation by pi about the x axis: (th, ph) -> (pi - th, -ph)
    ds3 = oracle.delta_seff(m, np.pi - th, -ph, o, np.pi - tn, -pn)
    assert abs(ds - ds3) < 1e-11


@pytest.mark.parametrize("beta", [0.05, 0.2, 1.0, 5.0])
def test_dseff_tracks_exact_diagonalisation(beta):
    # Method-error envelope on 6^3 with M = 256: measured <= 6e-4 relative;
    # a sign, scale or index slip gives O(1) errors.
    L = 6
    m = oracle.Model(L=L, M=256, beta=beta)
    th, ph = synth.random_angles(m.N, 3)
    o, tn, pn = 7, 0.4, 5.0
    ex = ed.exact_dseff(L, th, ph, o, tn, pn, beta)
    ds = oracle.delta_seff(m, th, ph, o, tn, pn)
    assert abs(ds - ex) < 2e-3 * abs(ex)


def test_dseff_high_temperature_series():
    # mu = 0: S = -N log 2 - (beta^2/8) Tr H^2 + (beta^4/192) Tr H^4 + O(beta^6),
    # Delta Tr H^2 = t^2 sum_d (S'_o - S_o).S_d.
    L, beta = 6, 0.05
    m = oracle.Model(L=L, M=256, beta=beta)
    th, ph = synth.random_angles(m.N, 3)
    o, tn, pn = 7, 0.4, 5.0
    S = lambda t, p: np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
    d2 = sum((S(tn, pn) - S(th[o], ph[o])) @ S(th[n], ph[n]) for n in oracle.start_sites(L, o)[1:])
    th2, ph2 = th.copy(), ph.copy()
    th2[o], ph2[o] = tn, pn
    tr4 = lambda A: np.trace(np.linalg.matrix_power(A, 4)).real
    d4 = tr4(ed.hamiltonian(L, th2, ph2)) - tr4(ed.hamiltonian(L, th, ph))
    series = -(beta ** 2 / 8) * d2 + (beta ** 4 / 192) * d4
    ds = oracle.delta_seff(m, th, ph, o, tn, pn)
    assert abs(ds - series) < 1e-3 * abs(series)


# --------------------------------------------------- Monte Carlo ----
def test_metropolis_rule_and_forcing():
    m = oracle.Model(L=2, M=32, beta=20.0, seed=3)
    th, ph = synth.random_angles(m.N, 1)
    for idx in range(12):
        t0, p0 = th.copy(), ph.copy()
        rec = oracle.step(m, th, ph, idx)
        own = 1 if (rec.dseff <= 0 or rec.u < math.exp(-rec.dseff)) else 0
        assert rec.own == own == rec.accepted
        site, tn, pn, u = oracle.propose(m, t0, p0, idx)
        assert (site, tn, pn, u) == (rec.site, rec.theta_new, rec.phi_new, rec.u)
        if rec.accepted:
            assert th[site] == tn and ph[site] == pn
        else:
            assert np.array_equal(th, t0)
    t0, p0 = th.copy(), ph.copy()
    rec = oracle.step(m, th, ph, 99, force=0)
    assert rec.accepted == 0 and np.array_equal(th, t0)
    rec = oracle.step(m, th, ph, 99, force=1)
    assert rec.accepted == 1 and th[rec.site] == rec.theta_new


def test_proposal_site_and_angles_from_the_counter():
    m = oracle.Model(L=4, seed=77, chain_id=5)
    th, ph = synth.random_angles(m.N, 2)
    for idx in [0, 1, 63, 10**6]:
        r = oracle.philox((idx, 1, 0, 0), (77, 5))
        site, tn, pn, u = oracle.propose(m, th, ph, idx)
        assert site == (r[0] * 64) >> 64
        assert abs(math.cos(tn) - (1 - 2 * oracle.u01(r[1]))) < 1e-15
        assert pn == 2 * math.pi * oracle.u01(r[2]) and u == oracle.u01(r[3])


def test_cone_proposal_stays_in_the_cap():
    c = 0.3
    m = oracle.Model(L=4, proposal=1, cone=c, seed=9)
    th, ph = synth.random_angles(m.N, 6)
    S = lambda t, p: np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
    cosines = []
    for idx in range(400):
        o, tn, pn, _ = oracle.propose(m, th, ph, idx)
        ca = S(th[o], ph[o]) @ S(tn, pn)
        r = oracle.philox((idx, 1, 0, 0), (9, 0))
        assert abs(ca - (1 - (1 - math.cos(c)) * oracle.u01(r[1]))) < 1e-12
        assert 0 <= tn <= math.pi and 0 <= pn < 2 * math.pi
        cosines.append(ca)
    assert min(cosines) >= math.cos(c) - 1e-12


def test_spin_initialisation():
    m = oracle.Model(L=16, seed=42)
    th, ph = oracle.init_spins(m, 2, 0.1)
    assert (th != 0).sum() == 409 == math.floor(0.1 * 4096)
    thf, phf = oracle.init_spins(m, 1)
    assert np.all(thf == 0) and np.all(phf == 0)
    thr, phr = oracle.init_spins(m, 0)
    r = oracle.philox((100, 2, 0, 0), (42, 0))
    assert abs(math.cos(thr[100]) - (1 - 2 * oracle.u01(r[0]))) < 1e-15
    assert abs(np.cos(thr).mean()) < 0.05 and abs(np.cos(phr).mean()) < 0.05
    # the randomised sites of the FM start carry the same per-site draws
    sel = th != 0
    assert np.array_equal(th[sel], thr[sel]) and np.array_equal(ph[sel], phr[sel])


def test_sweep_resume_is_bit_exact():
    m = oracle.Model(L=2, M=32, beta=10.0, seed=5)
    th, ph = synth.random_angles(m.N, 7)
    a_th, a_ph = th.copy(), ph.copy()
    mag2, acc2 = oracle.sweep(m, a_th, a_ph, 0, 2)
    b_th, b_ph = th.copy(), ph.copy()
    mag_a, acc_a = oracle.sweep(m, b_th, b_ph, 0, 1)
    mag_b, acc_b = oracle.sweep(m, b_th, b_ph, 1, 1)
    assert np.array_equal(a_th, b_th) and np.array_equal(a_ph, b_ph)
    assert acc2 == acc_a + acc_b and mag2[1] == mag_b[0]
    assert abs(oracle.magnetization(2, *synth.ferro_angles(8)) - 1.0) < 1e-15


# ------------------------------------------------- mixed start vectors ----
def test_mixed_vector_moments_match_exact_diagonalisation():
    # <a|T_n(Ht)|a> for a = o, v, o+v, o+iv from eigenvectors of the spinor-built
    # H, with |v> = (H' - H)|o> from two full Hamiltonians
    L, M = 4, 96
    m = oracle.Model(L=L, M=M)
    th, ph = synth.random_angles(m.N, 23)
    o, tn, pn = 21, 2.3, 4.1
    th2, ph2 = th.copy(), ph.copy()
    th2[o], ph2[o] = tn, pn
    v = (ed.hamiltonian(L, th2, ph2) - ed.hamiltonian(L, th, ph))[:, o]
    eo = np.zeros(m.N, complex)
    eo[o] = 1.0
    e, U = np.linalg.eigh(ed.hamiltonian(L, th, ph) / m.scale_a())
    T = np.cos(np.arange(M)[:, None] * np.arccos(np.clip(e, -1, 1))[None, :])
    got = oracle.mixed_moments(m, th, ph, o, tn, pn)
    for s, a in enumerate([eo, v, eo + v, eo + 1j * v]):
        w = np.abs(a.conj() @ U) ** 2                   # |<a|l>|^2
        assert np.abs(got[s] - T @ w).max() < 1e-12, s
    assert np.abs(got.imag).max() < 1e-13


def test_mixed_vector_moments_are_the_polarised_site_moments():
    # linearity: mu^{o+v} = mu^oo + mu^vv + 2 Re mu^ov, mu^{o+iv} = mu^oo + mu^vv - 2 Im mu^ov,
    # with mu^ov contracted from the 7x7 site moments (a separate recursion)
    L, M = 4, 128
    m = oracle.Model(L=L, M=M)
    th, ph = synth.random_angles(m.N, 24)
    o, tn, pn = 50, 0.7, 1.9
    c = oracle.contract(oracle.moments(m, th, ph, o), oracle.deltas(m, th, ph, o, tn, pn))
    oo, ov, vv = c[0].real, c[1], c[3].real
    got = oracle.mixed_moments(m, th, ph, o, tn, pn).real
    assert np.abs(got[0] - oo).max() < 1e-12
    assert np.abs(got[1] - vv).max() < 1e-12
    assert np.abs(got[2] - (oo + vv + 2 * ov.real)).max() < 1e-12
    assert np.abs(got[3] - (oo + vv - 2 * ov.imag)).max() < 1e-12


@pytest.mark.parametrize("kernel,K", [(0, 0), (1, 0), (0, 256)])
def test_mixed_vector_delta_seff_equals_site_vector_form(kernel, K):
    # the paper's G_ov / G_vo from mixed diagonal elements give the same Delta S
    # as the cross moments (exact up to rounding); a sign slip in either formula
    # changes Delta S at O(1)
    m = oracle.Model(L=4, M=128, K=K, beta=20.0, kernel=kernel)
    th, ph = synth.random_angles(m.N, 25)
    for o, tn, pn in [(5, 2.0, 0.3), (33, 0.2, 5.5), (60, 3.0, 2.0)]:
        ref = oracle.delta_seff(m, th, ph, o, tn, pn)
        got = oracle.delta_seff_mixed(m, th, ph, o, tn, pn)
        assert abs(got - ref) < 1e-11 * max(1.0, abs(ref)), (o, got, ref)
    assert oracle.delta_seff_mixed(m, th, ph, 12, th[12], ph[12]) == 0.0


# --------------------------------------- damping kernel and energy grid ----
def test_jackson_beats_lorentz_and_finer_grid_helps_at_large_m():
    # Method fidelity against ED on 6^3 (beta = 20): the Jackson kernel closes
    # the phase at the band top and tracks ED several times better than Lorentz
    # (lambda = 4), whose phase stays open by ~0.2-0.3 rad; K = 4M sharpens the
    # Jackson integral once M resolves the spectrum (M = 1024)
    L, beta = 6, 20.0
    th, ph = synth.random_angles(L ** 3, 1)
    props = [(17, 0.6, 2.0), (150, 2.5, 4.4)]
    ex = [ed.exact_dseff(L, th, ph, o, tn, pn, beta) for o, tn, pn in props]

    def err(M, K, kernel):
        m = oracle.Model(L=L, M=M, K=K, beta=beta, kernel=kernel)
        e, top = 0.0, 0.0
        for (o, tn, pn), x in zip(props, ex):
            ds, t = oracle.delta_seff(m, th, ph, o, tn, pn, with_phase_top=True)
            e, top = max(e, abs(ds - x)), max(top, abs(t))
        return e, top
    ej, tj = err(256, 0, 0)
    el, tl = err(256, 0, 1)
    assert tj < 1e-4 and tl > 0.1
    assert ej < 0.5 * el
    e1, _ = err(1024, 0, 0)
    e4, _ = err(1024, 4096, 0)
    assert e4 < 0.5 * e1


# ----------------------------------------------------- regression fixture ----
def test_oracle_reproduces_its_frozen_trajectory():
    # not a pin: guards the oracle against unnoticed changes of its arithmetic
    # (tests/golden/make_golden.py wrote the file from the oracle alone)
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_trajectory_4cubed.json")
    ref = json.load(open(path))
    m = oracle.Model(L=ref["lattice"], M=ref["M"], beta=ref["beta"], seed=ref["seed"],
                     chain_id=ref["chain_id"])
    th, ph = oracle.init_spins(m, 0)
    for rp in ref["proposals"]:
        r = oracle.step(m, th, ph, rp["index"])
        assert (r.site, r.u, r.theta_new, r.phi_new, r.accepted) == \
            (rp["site"], rp["u"], rp["theta_new"], rp["phi_new"], rp["accepted"])
        assert abs(r.dseff - rp["dseff"]) < 1e-12
    assert abs(oracle.magnetization(4, th, ph) - ref["magnetization"]) < 1e-14


def test_magnetization_closed_forms():
    # |sum_i S_i| / N for configurations with a known result
    L = 4
    N = L ** 3
    half = np.arange(N) < N // 2
    assert abs(oracle.magnetization(L, np.full(N, np.pi / 2), np.zeros(N)) - 1.0) < 1e-15
    assert abs(oracle.magnetization(L, np.full(N, np.pi / 2), np.full(N, np.pi / 2)) - 1.0) < 1e-15
    assert abs(oracle.magnetization(L, np.where(half, 0.0, np.pi), np.zeros(N))) < 1e-15
    assert abs(oracle.magnetization(L, np.full(N, np.pi / 2), np.where(half, 0.0, np.pi / 2))
               - math.sqrt(0.5)) < 1e-15
    ring = 2 * np.pi * np.arange(N) / N
    assert abs(oracle.magnetization(L, np.full(N, np.pi / 2), ring)) < 1e-14


@pytest.mark.parametrize("t,a", [(0.7, 0.0), (0.7, 8.0), (1.3, 9.5)])
def test_moments_hopping_scale_and_rescaling(t, a):
    # moments of Ht = H/a with H = -t t_ij for t != 1 and explicit a (a = 0
    # means the default 6t/(1 - 0.01)): the spinor-built H times t, divided
    # by the same a, diagonalised
    L, M = 4, 96
    m = oracle.Model(L=L, M=M, t=t, a=a)
    th, ph = synth.random_angles(m.N, 29)
    o = 18
    s = oracle.start_sites(L, o)
    ref = ed.cheb_moments_ed(ed.hamiltonian(L, th, ph, t) / m.scale_a(), s, s, M)
    assert np.abs(oracle.moments(m, th, ph, o) - ref).max() < 1e-12
    assert (m.scale_a() == a) if a else abs(m.scale_a() - 6 * t / 0.99) < 1e-15
