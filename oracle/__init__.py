"""Plain FP64 CPU oracle of the GFMC method (ctypes wrapper of gfmc_oracle.c).

TEST INFRASTRUCTURE ONLY.  This package is the correctness reference for the
HIP library; only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import it.  It never imports the HIP package and the
HIP package never imports it.

Every function forwards to one function of ``gfmc_oracle.c``; the paper
passage each one follows is cited there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gfmc_oracle.c")
# GFMC_ORACLE_LIB names an already built library to load instead (the pins'
# mutation test loads deliberately broken copies this way); build() then
# leaves it alone.
_LIB = os.environ.get("GFMC_ORACLE_LIB") or os.path.join(_HERE, "libgfmc_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, single-threaded)."""
    if os.environ.get("GFMC_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("t", ctypes.c_double), ("beta", ctypes.c_double),
        ("mu", ctypes.c_double), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
        ("kernel", ctypes.c_int32), ("lam", ctypes.c_double), ("a", ctypes.c_double),
        ("b", ctypes.c_double), ("proposal", ctypes.c_int32), ("cone", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("chain_id", ctypes.c_uint64),
    ]


class Record(ctypes.Structure):
    _fields_ = [
        ("index", ctypes.c_int64), ("site", ctypes.c_int32), ("own", ctypes.c_int32),
        ("accepted", ctypes.c_int32), ("theta_old", ctypes.c_double),
        ("phi_old", ctypes.c_double), ("theta_new", ctypes.c_double),
        ("phi_new", ctypes.c_double), ("dseff", ctypes.c_double), ("u", ctypes.c_double),
        ("phase_top", ctypes.c_double),
    ]


@dataclass
class Model:
    """Model and method parameters (defaults: the readings listed in the oracle)."""
    L: int
    t: float = 1.0
    beta: float = 20.0
    mu: float = 0.0
    M: int = 256
    K: int = 0              # 0 -> K = M
    kernel: int = 0         # 0 Jackson, 1 Lorentz
    lam: float = 4.0
    a: float = 0.0          # 0 -> 6 t / (1 - 0.01)
    b: float = 0.0
    proposal: int = 0       # 0 sphere, 1 cap
    cone: float = 0.3
    seed: int = 0
    chain_id: int = 0

    @property
    def N(self) -> int:
        return self.L ** 3

    def scale_a(self) -> float:
        return self.a if self.a > 0 else 6.0 * self.t / (1.0 - 0.01)

    def c(self) -> Params:
        return Params(self.L, self.t, self.beta, self.mu, self.M, self.K if self.K > 0 else self.M,
                      self.kernel, self.lam, self.scale_a(), self.b, self.proposal, self.cone,
                      self.seed & (2**64 - 1), self.chain_id & (2**64 - 1))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, i64, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        dp = P(d)
        sig = {
            "orc_philox4x64_10": (None, [P(u64), P(u64), P(u64)]),
            "orc_mulhi_index": (i64, [u64, i64]),
            "orc_u01": (d, [u64]),
            "orc_neighbor": (i32, [i32, i32, i32]),
            "orc_hopping": (None, [d, d, d, d, dp]),
            "orc_dense_ht": (None, [P(Params), dp, dp, dp]),
            "orc_start_sites": (None, [i32, i32, P(i32)]),
            "orc_moments": (None, [P(Params), dp, dp, i32, dp]),
            "orc_deltas": (None, [P(Params), dp, dp, i32, d, d, dp]),
            "orc_contract": (None, [i32, dp, dp, dp]),
            "orc_kernel_coeffs": (None, [i32, i32, d, dp]),
            "orc_green": (None, [i32, i32, dp, dp, dp]),
            "orc_det": (None, [i32, d, dp, dp, dp, dp, dp]),
            "orc_phase": (None, [i32, dp, dp]),
            "orc_quadrature": (d, [i32, d, d, d, d, dp]),
            "orc_delta_seff": (d, [P(Params), dp, dp, i32, d, d, dp]),
            "orc_mixed_moments": (None, [P(Params), dp, dp, i32, d, d, dp]),
            "orc_delta_seff_mixed": (d, [P(Params), dp, dp, i32, d, d, dp]),
            "orc_propose": (None, [P(Params), dp, dp, i64, P(i32), dp, dp, dp]),
            "orc_step": (None, [P(Params), dp, dp, i64, i32, P(Record)]),
            "orc_sweep": (i64, [P(Params), dp, dp, i64, i32, dp]),
            "orc_magnetization": (d, [i32, dp, dp]),
            "orc_init_spins": (None, [P(Params), i32, d, dp, dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cplx_view(a: np.ndarray) -> np.ndarray:
    return a.view(np.complex128)


# ---------------------------------------------------------------- RNG ----
def philox(ctr, key) -> list[int]:
    c = (ctypes.c_uint64 * 4)(*[int(x) & (2**64 - 1) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) & (2**64 - 1) for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def mulhi_index(r: int, n: int) -> int:
    return int(lib().orc_mulhi_index(r, n))


def u01(r: int) -> float:
    return float(lib().orc_u01(r))


# -------------------------------------------------------------- model ----
def neighbor(L: int, i: int, d: int) -> int:
    return int(lib().orc_neighbor(L, i, d))


def hopping(th_i, ph_i, th_j, ph_j) -> complex:
    o = np.zeros(2)
    lib().orc_hopping(th_i, ph_i, th_j, ph_j, _dp(o))
    return complex(o[0], o[1])


def dense_ht(m: Model, th: np.ndarray, ph: np.ndarray) -> np.ndarray:
    out = np.zeros((m.N, m.N, 2))
    p = m.c()
    lib().orc_dense_ht(ctypes.byref(p), _dp(th), _dp(ph), _dp(out))
    return _cplx_view(out)[..., 0]


def start_sites(L: int, o: int) -> list[int]:
    s = (ctypes.c_int32 * 7)()
    lib().orc_start_sites(L, o, s)
    return list(s)


def moments(m: Model, th: np.ndarray, ph: np.ndarray, o: int) -> np.ndarray:
    """mu[n, j, k] complex, shape (M, 7, 7)."""
    out = np.zeros((m.M, 7, 7, 2))
    p = m.c()
    lib().orc_moments(ctypes.byref(p), _dp(th), _dp(ph), o, _dp(out))
    return _cplx_view(out)[..., 0]


def deltas(m: Model, th, ph, o, th_new, ph_new) -> np.ndarray:
    out = np.zeros((6, 2))
    p = m.c()
    lib().orc_deltas(ctypes.byref(p), _dp(th), _dp(ph), o, th_new, ph_new, _dp(out))
    return _cplx_view(out)[..., 0]


def contract(mu: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """(M,7,7) complex moments, (6,) complex deltas -> (4, M): oo, ov, vo, vv."""
    M = mu.shape[0]
    mu_r = np.ascontiguousarray(np.stack([mu.real, mu.imag], -1))
    dl = np.ascontiguousarray(np.stack([delta.real, delta.imag], -1))
    out = np.zeros((4, M, 2))
    lib().orc_contract(M, _dp(mu_r), _dp(dl), _dp(out))
    return _cplx_view(out)[..., 0]


def kernel_coeffs(M: int, kind: int = 0, lam: float = 4.0) -> np.ndarray:
    g = np.zeros(M)
    lib().orc_kernel_coeffs(M, kind, lam, _dp(g))
    return g


def green(mu: np.ndarray, g: np.ndarray, K: int) -> np.ndarray:
    M = mu.shape[0]
    mu_r = np.ascontiguousarray(np.stack([mu.real, mu.imag], -1).astype(np.float64))
    out = np.zeros((K, 2))
    lib().orc_green(M, K, _dp(mu_r), _dp(np.ascontiguousarray(g, dtype=np.float64)), _dp(out))
    return _cplx_view(out)[..., 0]


def det(a: float, Goo, Gov, Gvo, Gvv) -> np.ndarray:
    K = len(Goo)

    def r(x):
        return np.ascontiguousarray(np.stack([np.real(x), np.imag(x)], -1).astype(np.float64))
    out = np.zeros((K, 2))
    lib().orc_det(K, a, _dp(r(Goo)), _dp(r(Gov)), _dp(r(Gvo)), _dp(r(Gvv)), _dp(out))
    return _cplx_view(out)[..., 0]


def phase(d: np.ndarray) -> np.ndarray:
    K = len(d)
    dr = np.ascontiguousarray(np.stack([d.real, d.imag], -1))
    phi = np.zeros(K)
    lib().orc_phase(K, _dp(dr), _dp(phi))
    return phi


def quadrature(K, beta, mu, a, b, phi: np.ndarray) -> float:
    return float(lib().orc_quadrature(K, beta, mu, a, b, _dp(np.ascontiguousarray(phi))))


def delta_seff(m: Model, th, ph, o, th_new, ph_new, with_phase_top=False):
    p = m.c()
    top = np.zeros(1)
    ds = float(lib().orc_delta_seff(ctypes.byref(p), _dp(th), _dp(ph), o, th_new, ph_new,
                                    _dp(top)))
    return (ds, float(top[0])) if with_phase_top else ds


def mixed_moments(m: Model, th, ph, o, th_new, ph_new):
    """Diagonal moments <a|T_n(Ht)|a> of the paper's mixed start vectors
    a = |o>, |v>, |o>+|v>, |o>+i|v>: complex array [4, M]."""
    p = m.c()
    mu = np.zeros((4, m.M, 2))
    lib().orc_mixed_moments(ctypes.byref(p), _dp(th), _dp(ph), o, th_new, ph_new, _dp(mu))
    return mu[..., 0] + 1j * mu[..., 1]


def delta_seff_mixed(m: Model, th, ph, o, th_new, ph_new, with_phase_top=False):
    """Delta S_eff with G_ov, G_vo from the mixed diagonal Green's functions."""
    p = m.c()
    top = np.zeros(1)
    ds = float(lib().orc_delta_seff_mixed(ctypes.byref(p), _dp(th), _dp(ph), o, th_new, ph_new,
                                          _dp(top)))
    return (ds, float(top[0])) if with_phase_top else ds


def propose(m: Model, th, ph, index: int):
    p = m.c()
    site = ctypes.c_int32()
    tn, pn, u = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_propose(ctypes.byref(p), _dp(th), _dp(ph), index, ctypes.byref(site),
                      ctypes.byref(tn), ctypes.byref(pn), ctypes.byref(u))
    return site.value, tn.value, pn.value, u.value


def step(m: Model, th, ph, index: int, force: int = -1) -> Record:
    """One proposal; th/ph are updated in place."""
    p = m.c()
    rec = Record()
    lib().orc_step(ctypes.byref(p), _dp(th), _dp(ph), index, force, ctypes.byref(rec))
    return rec


def sweep(m: Model, th, ph, sweep0: int, nsweeps: int):
    p = m.c()
    mag = np.zeros(max(nsweeps, 1))
    acc = lib().orc_sweep(ctypes.byref(p), _dp(th), _dp(ph), sweep0, nsweeps, _dp(mag))
    return mag[:nsweeps], int(acc)


def magnetization(L: int, th, ph) -> float:
    return float(lib().orc_magnetization(L, _dp(th), _dp(ph)))


def init_spins(m: Model, mode: int, frac: float = 0.0):
    th = np.zeros(m.N)
    ph = np.zeros(m.N)
    p = m.c()
    lib().orc_init_spins(ctypes.byref(p), mode, frac, _dp(th), _dp(ph))
    return th, ph
