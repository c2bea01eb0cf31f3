"""Pins of the oracle's adjoint (gradient of L = 1/2 ||u_nt - u_obs||^2 with
respect to u0 and the wave-speed coefficients) against facts that do not
come from the oracle's adjoint code: the transpose identities <A v, w> =
<v, A^T w>, a closed form for constant speed, finite differences of the
forward oracle, exact-GMRES limits and the MGRIT invariants."""
import dataclasses

import numpy as np
import pytest

from paper_2203_13382_amd import inputs as I
from paper_2203_13382_amd import workloads as W


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 3), (1, 5), (2, 1), (2, 3), (2, 5)])
def test_interp_transpose_identity(oracle, dim, p):
    """<S v, w> = <v, S^T w> for departure points anywhere (large, negative,
    exactly on nodes)."""
    nx = 10
    S = nx ** dim
    r = _rng(dim * 10 + p)
    h = 2.0 / nx
    xi = -1 + (np.arange(S) % nx) * h - r.uniform(-7.3, 7.3, S) * h
    xi[:3] = -1 + np.array([0, 4, 9]) * h            # on nodes (eps = 0)
    eta = None if dim == 1 else -1 + (np.arange(S) // nx) * h - r.uniform(-5, 5, S) * h
    v, w = r.standard_normal(S), r.standard_normal(S)
    Sv = oracle.interp(dim, nx, p, xi, eta, v)
    STw = oracle.interp_T(dim, nx, p, xi, eta, w)
    assert abs(Sv @ w - v @ STw) < 1e-12 * np.abs(Sv).sum() * np.abs(w).max()
    # column sums of S^T = row sums of S = 1 (weights sum to one)
    assert np.allclose(oracle.interp_T(dim, nx, p, xi, eta, np.ones(S)).sum(), S)


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 3), (2, 3), (2, 5)])
def test_B_transpose_and_exact_solve(oracle, dim, p):
    """<B v, w> = <v, B^T w>; GMRES with a Krylov space as large as the system
    solves B^T y = b exactly."""
    nx = 8 if dim == 1 else 3
    S = nx ** dim
    r = _rng(3 + p)
    sx = r.uniform(-0.05, 0.02, S)
    sy = None if dim == 1 else r.uniform(-0.05, 0.02, S)
    v, w = r.standard_normal(S), r.standard_normal(S)
    Bv = oracle.apply_B(dim, nx, p, sx, sy, v)
    BTw = oracle.apply_BT(dim, nx, p, sx, sy, w)
    assert abs(Bv @ w - v @ BTw) < 1e-12 * (np.abs(Bv @ w) + 1)
    y, it = oracle.bsolve_T(dim, nx, p, sx, sy, w, 10, 0.0)
    # exact up to one-pass Gram-Schmidt's loss of orthogonality, which enters
    # the Pythagorean norm once the Krylov space fills the system (S <= 10)
    assert np.abs(oracle.apply_BT(dim, nx, p, sx, sy, y) - w).max() < 1e-8


def test_coarse_operator_transpose(oracle):
    """<Phi_l v, w> = <v, Phi_l^T w> on every level when GMRES is exact
    (nx = 8 <= kmax)."""
    pr = W.Problem(1, 8, 32, 1.7 * 2 / 8, 3, 3, W.alpha_cfg12(0.6))
    sv = W.Solver(m=[4, 2], coarsest_max_points=2, gmres_rtol=0.0, gmres_kmax=10)
    ctx = oracle.Context(pr, sv)
    r = _rng(9)
    for l in range(ctx.L):
        for n in (0, ctx.N[l] - 1):
            v, w = r.standard_normal(8), r.standard_normal(8)
            a = ctx.apply_phi(l, n, v) @ w
            b = v @ ctx.apply_phi_T(l, n, w)
            assert abs(a - b) < 1e-9 * (abs(a) + 1), (l, n)


def test_constant_integer_cfl_closed_form(oracle):
    """alpha = 1 and dt = 2h: every step shifts by two nodes, S^T shifts back,
    so lambda_0 is lamT shifted by -2 nt nodes."""
    nx, nt = 16, 5
    pr = W.Problem(1, nx, nt, 2 * 2.0 / nx, 3, 3, [W.term(1.0)])
    lamT = _rng(1).standard_normal(nx)
    lam = oracle.adjoint_seq(pr, lamT)
    assert np.allclose(lam[0], np.roll(lamT, -2 * nt), atol=1e-14)


def test_weight_derivatives_match_differences(oracle):
    for p in (1, 3, 5):
        for eps in (0.0, 0.1, 0.45, 0.9):
            d = 1e-6
            fd = (oracle.weights(p, eps + d) - oracle.weights(p, eps - d)) / (2 * d) if eps > 0 else \
                (oracle.weights(p, eps + d) - oracle.weights(p, eps)) / d
            assert np.abs(oracle.weights_deps(p, eps) - fd).max() < (1e-8 if eps > 0 else 1e-5)


@pytest.mark.parametrize("dim", [1, 2])
def test_erk_tangent_matches_differences(oracle, dim):
    if dim == 1:
        pr = W.Problem(1, 16, 4, 0.1, 3, 3, [W.term(1.0), W.term(0.5, kx=1.0, px=-np.pi / 2, kt=2.0)])
    else:
        a, b = W.field_cfg5((1.0, 0.3, 0.8, 0.2))
        pr = W.Problem(2, 16, 4, 0.1, 3, 5, a, b)
    x, y, t, dt = 0.3, -0.4, 0.7, 0.13
    dxi, deta = oracle.erk_back_tangent(pr, x, y, t, dt)
    nq = len(dxi)
    for q in range(nq):
        d = 1e-6

        def shifted(s):
            al = [tuple(v + (s if (k == q and j == 0) else 0.0) for j, v in enumerate(term))
                  for k, term in enumerate(pr.alpha)]
            be = [tuple(v + (s if (len(pr.alpha) + k == q and j == 0) else 0.0) for j, v in enumerate(term))
                  for k, term in enumerate(pr.beta or [])]
            return dataclasses.replace(pr, alpha=al, beta=be)
        xp, yp = oracle.erk_back(shifted(d), x, y, t, dt)
        xm, ym = oracle.erk_back(shifted(-d), x, y, t, dt)
        assert abs(dxi[q] - (xp - xm) / (2 * d)) < 1e-9, q
        if dim == 2:
            assert abs(deta[q] - (yp - ym) / (2 * d)) < 1e-9, q


def _perturbed(pr, q, s):
    na = len(pr.alpha)
    al = [tuple(v + (s if (k == q and j == 0) else 0.0) for j, v in enumerate(t)) for k, t in enumerate(pr.alpha)]
    be = [tuple(v + (s if (na + k == q and j == 0) else 0.0) for j, v in enumerate(t))
          for k, t in enumerate(pr.beta or [])]
    return dataclasses.replace(pr, alpha=al, beta=be)


def _loss(oracle, pr, u0, u_obs):
    u = oracle.seq_fine(pr, u0)
    r = u[-1] - u_obs
    return 0.5 * float(r @ r)


@pytest.mark.parametrize("dim", [1, 2])
def test_gradient_matches_central_differences(oracle, dim):
    """dL/dtheta and dL/du0 (along random directions) against central
    differences of the forward oracle with step 1e-6.  The interpolant is
    only piecewise smooth in the departure point (its slope jumps at mesh
    nodes), so the coefficients are generic: at theta = (1, 0, 1, 0) some
    departure points sit exactly on nodes and a central difference averages
    two one-sided slopes."""
    if dim == 1:
        pr = W.Problem(1, 32, 24, 1.3 * 2 / 32, 3, 3, W.alpha_cfg12(0.5))
    else:
        a, b = W.field_cfg5((1.0, 0.3, 0.9, 0.2))
        pr = W.Problem(2, 12, 8, 2.0 * 2 / 12, 3, 3, a, b)
    u0 = I.initial_condition(pr, 0)
    obs_pr = _perturbed(_perturbed(pr, 0, 0.07), 1, -0.04)
    u_obs = oracle.seq_fine(obs_pr, u0)[-1]
    L0, g_u0, g_th = oracle.loss_and_gradient(pr, u0, u_obs)
    assert L0 > 0
    d = 1e-6
    for q in range(len(g_th)):
        fd = (_loss(oracle, _perturbed(pr, q, d), u0, u_obs) - _loss(oracle, _perturbed(pr, q, -d), u0, u_obs)) / (2 * d)
        assert abs(g_th[q] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g_th).max()), (q, g_th[q], fd)
    r = _rng(5)
    for _ in range(4):
        e = r.standard_normal(u0.size)
        e /= np.linalg.norm(e)
        fd = (_loss(oracle, pr, u0 + d * e, u_obs) - _loss(oracle, pr, u0 - d * e, u_obs)) / (2 * d)
        assert abs(g_u0 @ e - fd) <= 1e-7 * max(abs(fd), np.linalg.norm(g_u0))


def test_adjoint_mgrit_single_level_is_sequential(oracle):
    pr = W.Problem(1, 24, 16, 1.1 * 2 / 24, 3, 3, W.alpha_cfg12())
    sv = W.Solver(m=[4], max_levels=1)
    ctx = oracle.Context(pr, sv)
    lamT = _rng(2).standard_normal(pr.nx)
    mu, st, _ = ctx.mgrit_adjoint(lamT, np.zeros((pr.nt + 1, pr.nx)))
    lam = oracle.adjoint_seq(pr, lamT)
    assert np.array_equal(mu[::-1], lam)


@pytest.mark.parametrize("relax,levels", [("F", 2), ("FCF", 2), ("FCF", 9)])
def test_adjoint_mgrit_converges_to_sequential(oracle, relax, levels):
    """Converged adjoint MGRIT equals the sequential adjoint sweep; two-level
    F-relaxation is exact after nt/m cycles (the first k coarse intervals are
    exact after k cycles)."""
    pr = W.Problem(1, 32, 32, 1.6 * 2 / 32, 3, 3, W.alpha_cfg12(0.4))
    sv = W.Solver(m=[4], relax=relax, max_levels=levels, coarsest_max_points=2, gmres_rtol=1e-2,
                  tol=1e-12, tol_mode="rel", max_iter=40)
    ctx = oracle.Context(pr, sv)
    lamT = _rng(4).standard_normal(pr.nx)
    mu0 = np.zeros((pr.nt + 1, pr.nx))
    mu0[::4] = _rng(6).uniform(0, 1, (pr.nt // 4 + 1, pr.nx))
    mu, st, hist = ctx.mgrit_adjoint(lamT, mu0)
    lam = oracle.adjoint_seq(pr, lamT)
    assert st["status"] == "converged"
    assert np.abs(mu[::-1] - lam).max() < 1e-9 * np.abs(lam).max()
    assert np.all(np.diff(hist) < 0)
    if relax == "F" and levels == 2:
        assert st["iterations"] <= pr.nt // 4 + 1
