"""Seeded synthetic inputs shared by the GPU path and the test oracle.

This module draws random numbers and samples the initial condition on the
mesh; it holds none of the method's arithmetic.  Every draw comes from
``numpy.random.default_rng(seed)`` so both sides receive identical arrays.
"""
from __future__ import annotations

import numpy as np


def mesh(nx: int) -> np.ndarray:
    """Nodes x_i = -1 + i*h, h = 2/nx."""
    return -1.0 + np.arange(nx) * (2.0 / nx)


def fourier_ic_1d(nx: int, seed: int = 0, modes: int = 8) -> np.ndarray:
    """u0(x) = sum_{k=1}^{modes} (a_k cos k pi x + b_k sin k pi x)/k^2,
    a_k, b_k ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    ab = rng.standard_normal((modes, 2))
    x = mesh(nx)
    u = np.zeros(nx)
    for k in range(1, modes + 1):
        u += (ab[k - 1, 0] * np.cos(k * np.pi * x) + ab[k - 1, 1] * np.sin(k * np.pi * x)) / k**2
    return u


def fourier_ic_2d(nx: int, seed: int = 0, modes: int = 8) -> np.ndarray:
    """u0(x,y) = sum_{kx,ky=1}^{modes} (a cos pi(kx x+ky y) + b sin pi(kx x+ky y))
    /(kx^2+ky^2), a, b ~ N(0,1); flattened with x fastest."""
    rng = np.random.default_rng(seed)
    ab = rng.standard_normal((modes, modes, 2))
    x = mesh(nx)
    X, Y = np.meshgrid(x, x, indexing="xy")   # X[j, i] = x_i, Y[j, i] = y_j
    u = np.zeros((nx, nx))
    for kx in range(1, modes + 1):
        for ky in range(1, modes + 1):
            ph = np.pi * (kx * X + ky * Y)
            u += (ab[kx - 1, ky - 1, 0] * np.cos(ph) + ab[kx - 1, ky - 1, 1] * np.sin(ph)) / (kx * kx + ky * ky)
    return u.reshape(-1)


def initial_condition(pr, seed: int = 0) -> np.ndarray:
    return fourier_ic_1d(pr.nx, seed) if pr.dim == 1 else fourier_ic_2d(pr.nx, seed)


def initial_iterate(nt: int, S: int, m0: int, seed: int = 1, dtype=np.float64) -> np.ndarray:
    """Space-time initial iterate [(nt+1), S]: entries of the C-points
    (every m0-th time point) uniform in [0,1), the rest zero (MGRIT
    overwrites F-points before reading them)."""
    rng = np.random.default_rng(seed)
    u = np.zeros((nt + 1, S), dtype=dtype)
    nc = nt // m0 if m0 > 0 else nt
    step = m0 if m0 > 0 else 1
    u[::step][: nc + 1] = rng.random((nc + 1, S)).astype(dtype)
    return u


def batch_draws(n: int = 64, seed: int = 4):
    """Config-4 draws: nx in {256..8192} and nt in {1024..16384} (powers of
    two), p in {1,3,5}, alpha amplitude in [0.2, 0.8]."""
    rng = np.random.default_rng(seed)
    nx = 2 ** rng.integers(8, 14, size=n)
    nt = 2 ** rng.integers(10, 15, size=n)
    p = rng.choice([1, 3, 5], size=n)
    amp = rng.uniform(0.2, 0.8, size=n)
    return [dict(nx=int(a), nt=int(b), p=int(c), amp=float(d)) for a, b, c, d in zip(nx, nt, p, amp)]
