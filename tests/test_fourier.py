"""Pins of the two-level Fourier estimate (paper_2203_13382_amd/fourier.py,
eq. rho_MGRIT_asym, Figs. 2 and 3) against things it does not compute
itself: the oracle's operators applied to Fourier modes (for constant speed
they are circulant, so every mode is an eigenvector), the oracle's sigma,
the statements the paper makes about the estimate, and convergence factors
measured with the oracle's MGRIT."""
import numpy as np
import pytest

from paper_2203_13382_amd import fourier as F
from paper_2203_13382_amd import workloads as W


def _modes(nx):
    k = np.arange(nx)
    for f in range(nx):
        w = 2.0 * np.pi * f / nx
        yield w, np.cos(w * k), np.sin(w * k)


def _check_symbol(apply, sym, nx, tol):
    """apply(v) on cos/sin modes equals Re/Im of sym(w) * exp(i w k)."""
    for w, cv, sv in _modes(nx):
        s = complex(sym(np.array([w]))[0])
        assert np.abs(apply(cv) - (s.real * cv - s.imag * sv)).max() < tol, (w, s)
        assert np.abs(apply(sv) - (s.real * sv + s.imag * cv)).max() < tol, (w, s)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("c", [0.3, 0.85, 1.7, 4.25])
def test_sl_symbol_matches_oracle_step(oracle, p, c):
    nx = 16
    h = 2.0 / nx
    xi = -1.0 + np.arange(nx) * h - c * h          # exact departure points, alpha = 1
    _check_symbol(lambda v: oracle.interp(1, nx, p, xi, None, v), lambda w: F.sl_symbol(p, c, w), nx, 1e-12)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_dp1_symbol_matches_oracle(oracle, p):
    nx = 12
    _check_symbol(lambda v: oracle.apply_D(nx, p, v), lambda w: F.dp1_symbol(p, w) + 0j, nx, 1e-11)


@pytest.mark.parametrize("p", [1, 3, 5])
@pytest.mark.parametrize("c,m", [(0.85, 4), (0.6, 8), (1.3, 2), (2.2, 16)])
def test_phi_matches_oracle_sigma(oracle, p, c, m):
    """For constant speed the level-1 sigma of the method is the constant
    phi of eq. (varphi_p_def)."""
    nx = 16
    pr = W.Problem(1, nx, 4 * m, c * 2.0 / nx, p, p, [W.term(1.0)], [])
    ctx = oracle.Context(pr, W.Solver(m=[m], max_levels=2))
    sig = ctx.sigma(1)
    assert np.abs(sig - F.phi_two_level(p, c, m)).max() < 1e-12 * max(1.0, abs(sig).max())


@pytest.mark.parametrize("p", [1, 3])
@pytest.mark.parametrize("c,m", [(0.85, 4), (0.6, 8), (1.3, 2)])
def test_coarse_symbols_match_oracle(oracle, p, c, m):
    """mu(w) of the three coarse operators against the oracle's level-1 step with
    an exact linear solve (nx = 8, Krylov space of dimension 8)."""
    nx = 8
    for coarse in ("modified", "redisc", "fwd_euler"):
        pr = W.Problem(1, nx, 4 * m, c * 2.0 / nx, p, p, [W.term(1.0)], [])
        sv = W.Solver(m=[m], max_levels=2, gmres_kmax=10, gmres_rtol=0.0, coarse_op=coarse)
        ctx = oracle.Context(pr, sv)
        _check_symbol(lambda v: ctx.apply_phi(1, 0, v), lambda w: F.coarse_symbol(p, c, m, w, coarse), nx, 1e-10)


def test_paper_statements():
    """Sec. 2.3 and Sec. 3.2: the rediscretized operator has a CFL interval in
    [0.5, 1] with rho > 1 that grows with m (odd p) and rho > 1 almost
    everywhere for even p; the backward-Euler operator converges for every
    CFL number."""
    cs = np.linspace(0.5, 1.0, 51)[1:-1]
    for p in (1, 3):
        frac = [np.mean([F.rho(p, c, m, "redisc") > 1 for c in cs]) for m in (2, 4, 8, 16)]
        assert frac[0] > 0.1 and np.all(np.diff(frac) > 0), (p, frac)
    for p in (2, 4):
        for m in (2, 4, 8, 16):
            assert np.mean([F.rho(p, c, m, "redisc") > 1 for c in cs]) > 0.9, (p, m)
    for p in (1, 3):
        for m in (2, 4, 8, 16):
            r = [F.rho(p, c, m, "modified") for c in np.linspace(0.05, 4.0, 80)]
            assert max(r) < 1.0, (p, m, max(r))


def test_forward_euler_statements():
    """Sec. 3.2, case 1: for constant speed the forward-Euler correction
    I + phi D_{p+1} is stable for small m (|1 + phi d(w)| <= 1, and the
    estimate is below 1 for every CFL number) and unstable for larger m
    (norm above 1, the estimate above 1 for some CFL numbers)."""
    w = F.omegas()
    cs = np.linspace(0.05, 4.0, 80)
    for p in (1, 3):
        for m in (2, 4):
            assert max(np.abs(1 + F.phi_two_level(p, c, m) * F.dp1_symbol(p, w)).max() for c in cs) <= 1 + 1e-12
            assert max(F.rho(p, c, m, "fwd_euler") for c in cs) < 1
        for m in (8, 16):
            assert max(np.abs(1 + F.phi_two_level(p, c, m) * F.dp1_symbol(p, w)).max() for c in cs) > 1.5
            assert max(F.rho(p, c, m, "fwd_euler") for c in cs) > 1


@pytest.mark.parametrize("p,c,m,coarse", [(1, 0.8, 4, "modified"), (3, 0.8, 4, "modified"),
                                          (1, 0.8, 2, "fwd_euler"),
                                          (1, 0.9, 4, "redisc"), (1, 0.62, 2, "redisc")])
def test_estimate_matches_measured_factor(oracle, p, c, m, coarse):
    """Two-level FCF MGRIT with 10 GMRES iterations (rtol 0) on alpha = 1:
    the factor of the last cycles lies near the estimate (within 20% below,
    5% above), and above 1 where the estimate is."""
    nx, nt = 64, 2 ** 12
    pr = W.Problem(1, nx, nt, c * 2.0 / nx, p, p, [W.term(1.0)], [])
    sv = W.Solver(m=[m], max_levels=2, gmres_kmax=10, gmres_rtol=0.0, tol=1e-13, max_iter=40, coarse_op=coarse)
    ctx = oracle.Context(pr, sv)
    u0 = np.sin(np.pi * (-1.0 + np.arange(nx) * 2.0 / nx)) ** 4
    u, st, hist = ctx.mgrit(u0, np.random.default_rng(5).random((nt + 1, nx)))
    fac = hist[-1] / hist[-2]
    est = F.rho(p, c, m, coarse)
    assert 0.8 * est <= fac <= 1.05 * est, (fac, est)
    if est > 1:
        assert fac > 1
