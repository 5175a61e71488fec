"""Exact-diagonalisation helpers for the oracle pins (numpy only).

The Hamiltonian here is built from the spinor overlap <chi_i|chi_j> with
chi = (cos(theta/2) e^{-i phi/2}, sin(theta/2) e^{i phi/2}), a different formula
from the angle form the oracle writes out, so a slip in either shows up.
"""
import numpy as np

DIRS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def spinor(th, ph):
    return np.stack([np.cos(th / 2) * np.exp(-0.5j * ph), np.sin(th / 2) * np.exp(0.5j * ph)], -1)


def nbr(L, i, d):
    x, y, z = i % L, (i // L) % L, i // (L * L)
    dx, dy, dz = DIRS[d]
    return (x + dx) % L + L * (((y + dy) % L) + L * ((z + dz) % L))


def hamiltonian(L, th, ph, t=1.0):
    N = L ** 3
    H = np.zeros((N, N), complex)
    chi = spinor(np.asarray(th), np.asarray(ph))
    idx = np.arange(N)
    for d in range(6):
        j = nbr(L, idx, d)
        np.add.at(H, (idx, j), -t * np.einsum('is,is->i', chi.conj(), chi[j]))
    return H


def cheb_moments_ed(Ht, rows, cols, M):
    """<r|T_n(Ht)|c> for all n < M via eigen-decomposition."""
    e, U = np.linalg.eigh(Ht)
    T = np.cos(np.arange(M)[:, None] * np.arccos(np.clip(e, -1, 1))[None, :])
    return np.einsum('jl,nl,kl->njk', U[rows, :], T, U[cols, :].conj())


def exact_dseff(L, th, ph, o, tn, pn, beta, mu=0.0, t=1.0):
    th2, ph2 = np.array(th), np.array(ph)
    th2[o], ph2[o] = tn, pn
    e1 = np.linalg.eigvalsh(hamiltonian(L, th, ph, t))
    e2 = np.linalg.eigvalsh(hamiltonian(L, th2, ph2, t))
    S = lambda e: -np.sum(np.logaddexp(0.0, -beta * (e - mu)))
    return S(e2) - S(e1)
