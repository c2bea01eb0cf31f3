"""Fourier estimate of the two-level MGRIT convergence factor for the
constant-wave-speed problem (alpha = 1), as used for Figs. 2 and 3 of the
paper.

For constant speed, every fine semi-Lagrangian step is the same circulant
matrix, so it acts on the Fourier mode exp(i w k) by a factor lambda(w).  The
coarse operator acts by mu(w): the rediscretized step S(m dt) of Sec. 2.3,
the backward-Euler coarse operator of eq. (Bp_def),
[I - phi D_{p+1}]^{-1} S(m dt), or the forward-Euler one of eq. (Fp_def),
[I + phi D_{p+1}] S(m dt), with the constant phi of eq. (varphi_p_def)
and D_{p+1} the second-order central difference (delta^2)^{(p+1)/2}.  The
estimate of eq. (rho_MGRIT_asym) is
    rho(c) = max_w |lambda|^m |lambda^m - mu| / (1 - |mu|)
over 512 equispaced w in [-pi, pi), with c = dt/h the fine CFL number.

This is an analysis tool on the host (numpy); it is not part of the GPU
path and shares no code with it.
"""
from __future__ import annotations

from math import factorial

import numpy as np

N_OMEGA = 512


def omegas(n: int = N_OMEGA) -> np.ndarray:
    """n equispaced frequencies in [-pi, pi)."""
    return -np.pi + 2.0 * np.pi * np.arange(n) / n


def stencil_first(p: int, eps: float) -> int:
    """Offset of the westmost stencil node from the east neighbour x_E of the
    departure point (Sec. 2.1): symmetric for odd p; for even p the extra
    node goes west when eps > 1/2."""
    if p % 2:
        return -(p + 1) // 2
    return -(p // 2 + 1) if eps > 0.5 else -(p // 2)


def lagrange_weights(p: int, eps: float) -> np.ndarray:
    """Weights of the nodes x_E + (first + j) h, j = 0..p, for the departure
    point x_E - eps h (Lagrange basis evaluated at z = -eps - first)."""
    first = stencil_first(p, eps)
    z = -eps - first
    w = np.ones(p + 1)
    for j in range(p + 1):
        for k in range(p + 1):
            if k != j:
                w[j] *= (z - k) / (j - k)
    return w


def sl_symbol(p: int, d: float, w: np.ndarray) -> np.ndarray:
    """Symbol of the semi-Lagrangian step whose departure points lie d cells
    upwind of every node: u_new[i] = sum_j w_j u[i - floor(d) + first + j]."""
    fl = np.floor(d)
    eps = d - fl
    first = stencil_first(p, eps)
    wt = lagrange_weights(p, eps)
    return sum(wt[j] * np.exp(1j * w * (-fl + first + j)) for j in range(p + 1))


def dp1_symbol(p: int, w: np.ndarray) -> np.ndarray:
    """Symbol of D_{p+1} = (delta^2)^{(p+1)/2}, odd p."""
    return (2.0 * np.cos(w) - 2.0) ** ((p + 1) // 2)


def fpoly(p: int, z: float) -> float:
    """f_{p+1}(z) of eq. (fpoly_def), odd p: prod_{q=-l}^{r} (q + z) / (p+1)!
    with l = (p+1)/2, r = (p-1)/2."""
    l, r = (p + 1) // 2, (p - 1) // 2
    prod = 1.0
    for q in range(-l, r + 1):
        prod *= q + z
    return prod / factorial(p + 1)


def phi_two_level(p: int, c: float, m: int) -> float:
    """phi_{p+1} of eq. (varphi_p_def) for constant speed: every fine step has
    eps = frac(c), the coarse step eps_c = frac(m c)."""
    eps, eps_c = c - np.floor(c), m * c - np.floor(m * c)
    return (-1.0) ** (p + 1) * (fpoly(p, eps_c) - m * fpoly(p, eps))


def coarse_symbol(p: int, c: float, m: int, w: np.ndarray, coarse: str = "modified") -> np.ndarray:
    """mu(w): rediscretized S(m dt), the backward-Euler operator
    [I - phi D_{p+1}]^{-1} S(m dt) ('modified'), or the forward-Euler
    operator [I + phi D_{p+1}] S(m dt) ('fwd_euler')."""
    mu = sl_symbol(p, m * c, w)
    if coarse == "redisc":
        return mu
    if coarse == "fwd_euler":                  # eq. (Fp_def)
        return mu * (1.0 + phi_two_level(p, c, m) * dp1_symbol(p, w))
    if coarse != "modified":
        raise ValueError("coarse must be 'modified', 'fwd_euler' or 'redisc'")
    return mu / (1.0 - phi_two_level(p, c, m) * dp1_symbol(p, w))


def rho(p: int, c: float, m: int, coarse: str = "modified", n_omega: int = N_OMEGA) -> float:
    """Two-level estimate of eq. (rho_MGRIT_asym) at fine CFL number c."""
    w = omegas(n_omega)
    lam = sl_symbol(p, c, w)
    mu = coarse_symbol(p, c, m, w, coarse)
    num = np.abs(lam) ** m * np.abs(lam ** m - mu)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = num / (1.0 - np.abs(mu))
    # a mode propagated identically on both grids (w = 0: the mean) carries
    # no error; any other mode with |mu| >= 1 is not damped at all
    r = np.where(num <= 1e-14, 0.0, np.where(np.abs(mu) < 1.0, r, np.inf))
    return float(np.max(r))
