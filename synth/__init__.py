"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds no arithmetic of the method: only spin configurations and parameter grids
drawn with numpy's own generators, so that the oracle and the HIP library are fed
identical inputs without either depending on the other.
"""
from __future__ import annotations

import numpy as np


def random_angles(N: int, seed: int):
    """Directions uniform on the unit sphere: (theta, phi) float64 arrays."""
    g = np.random.default_rng(seed)
    cos_t = g.uniform(-1.0, 1.0, N)
    phi = g.uniform(0.0, 2.0 * np.pi, N)
    return np.arccos(cos_t), phi


def ferro_angles(N: int, theta: float = 0.0, phi: float = 0.0):
    return np.full(N, float(theta)), np.full(N, float(phi))


def canted_angles(N: int, seed: int, spread: float = 0.4):
    """Directions scattered around +z with polar angles up to `spread` (rad)."""
    g = np.random.default_rng(seed)
    return g.uniform(0.0, spread, N), g.uniform(0.0, 2.0 * np.pi, N)


def temperature_ladder(n: int, t_lo: float = 0.02, t_hi: float = 0.2):
    """n temperatures linearly spaced in [t_lo, t_hi] (units of t)."""
    if n == 1:
        return np.array([t_lo])
    return t_lo + (t_hi - t_lo) * np.arange(n) / (n - 1)
