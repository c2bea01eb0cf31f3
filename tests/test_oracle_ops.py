"""Pins of the oracle's vector operators.

* the semi-Lagrangian step is an exact periodic shift for constant speed at
  integer CFL and converges at rate O(h^{p+1}/dt) (Sec. 2.1);
* backtracking with a space-independent speed equals m fine ERK steps
  (footnote of Sec. 3.3.1; SM6 in 2D);
* phi for constant speed is the closed form of Sec. 3.2 (worked values);
* GMRES with a full Krylov space is a direct solve;
* Lemma 3.3 / SM1: the modified coarse operator matches the ideal one to
  O(h^{p+2}) while the plain coarse SL step matches it only to O(h^{p+1}).
"""
import math

import numpy as np
import pytest

from paper_2203_13382_amd import inputs as I
from paper_2203_13382_amd import workloads as W


def _prob(dim, nx, nt, cfl, p, r, alpha, beta=()):
    return W.Problem(dim, nx, nt, cfl * 2.0 / nx, p, r, list(alpha), list(beta))


# ------------------------------------------------------------ SL step
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_integer_cfl_is_exact_shift_1d(oracle, p):
    nx = 64
    pr = _prob(1, nx, 5, 4.0, p, 1, [W.term(1.0)])
    u0 = I.fourier_ic_1d(nx, 3)
    u = oracle.seq_fine(pr, u0)
    for n in range(1, 6):
        assert np.array_equal(u[n], np.roll(u0, 4 * n))


@pytest.mark.parametrize("p", [1, 3, 5])
def test_integer_cfl_is_exact_shift_2d(oracle, p):
    nx = 16
    pr = _prob(2, nx, 3, 2.0, p, 1, [W.term(1.0)], [W.term(-0.5)])  # shifts (+2, -1) cells
    u0 = I.fourier_ic_2d(nx, 3).reshape(nx, nx)
    u = oracle.seq_fine(pr, u0.reshape(-1))
    for n in range(1, 4):
        assert np.array_equal(u[n].reshape(nx, nx), np.roll(np.roll(u0, 2 * n, axis=1), -n, axis=0))


@pytest.mark.parametrize("p", [1, 3])
def test_sl_convergence_order_constant_speed(oracle, p):
    """u(x,T) = u0(x - alpha T); error O(dt^r + h^{p+1}/dt) with exact
    departure points and dt = 0.85 h gives O(h^p) (Sec. 2.1)."""
    errs = []
    for nx in (32, 64, 128):
        nt = nx // 2
        pr = _prob(1, nx, nt, 0.85, p, 1, [W.term(1.0)])
        x = I.mesh(nx)
        u0 = np.sin(math.pi * x) + 0.4 * np.cos(2 * math.pi * x)
        u = oracle.seq_fine(pr, u0)
        T = nt * pr.dt
        exact = np.sin(math.pi * (x - T)) + 0.4 * np.cos(2 * math.pi * (x - T))
        errs.append(np.abs(u[-1] - exact).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > p - 0.3, (errs, orders)


def test_sl_step_symbol_constant_speed(oracle):
    """Constant speed, non-integer CFL: S is circulant, so a Fourier mode is
    an eigenvector with eigenvalue the interpolation weights' symbol."""
    nx, p, c = 64, 3, 2.3
    pr = _prob(1, nx, 1, c, p, 1, [W.term(1.0)])
    (xi,) = oracle.depart_fine(pr, 0)
    h = pr.h
    x = I.mesh(nx)
    w = oracle.weights(p, c - math.floor(c))
    ell, rr = oracle.stencil(p, c - math.floor(c))
    omega = 5 * math.pi
    lam = sum(w[j + ell] * np.exp(1j * omega * h * (j - math.floor(c))) for j in range(-ell, rr + 1))
    for f, g in ((np.cos, lambda z: z.real), (np.sin, lambda z: z.imag)):
        out = oracle.interp(1, nx, p, xi, None, f(omega * x))
        ref = g(lam * np.exp(1j * omega * x))
        assert np.abs(out - ref).max() < 1e-13


@pytest.mark.parametrize("p", [1, 3, 5])
def test_interp_2d_reproduces_tensor_polynomials(oracle, p):
    """Tensor-product interpolation (Sec. 4.1) is exact for x^a y^b, a,b <= p,
    away from the periodic seam."""
    nx = 32
    h = 2.0 / nx
    rng = np.random.default_rng(1)
    S = nx * nx
    ii, jj = np.meshgrid(np.arange(nx), np.arange(nx), indexing="xy")
    xi = (-1 + ii * h - rng.uniform(-1.5, 1.5, (nx, nx)) * h).reshape(-1)
    eta = (-1 + jj * h - rng.uniform(-1.5, 1.5, (nx, nx)) * h).reshape(-1)
    X = (-1 + ii * h).reshape(-1)
    Y = (-1 + jj * h).reshape(-1)
    inner = ((ii > 6) & (ii < nx - 7) & (jj > 6) & (jj < nx - 7)).reshape(-1)
    for a in range(p + 1):
        for b in range(p + 1 - a):
            u = X ** a * Y ** b
            out = oracle.interp(2, nx, p, xi, eta, u)
            assert np.abs(out[inner] - (xi ** a * eta ** b)[inner]).max() < 1e-12
    assert S == u.size


# ------------------------------------------------------------ backtracking
@pytest.mark.parametrize("r", [1, 3, 5])
def test_backtrack_time_only_speed_equals_fine_steps_1d(oracle, r):
    """Footnote of Sec. 3.3.1: for a space-independent speed the backtracked
    coarse departure point equals m fine ERK steps of size dt."""
    nx, m, cfl = 64, 8, 0.85
    pr = _prob(1, nx, m, cfl, r, r, [W.term(1.0, kt=2.0), W.term(0.3)])
    fine = np.stack([oracle.depart_fine(pr, k)[0] for k in range(m)])
    c = oracle.backtrack_1d(nx, m, fine)
    x = I.mesh(nx)
    for i in range(0, nx, 7):
        xs = x[i]
        for k in range(m - 1, -1, -1):
            xs, _ = oracle.erk_back(pr, xs, 0.0, (k + 1) * pr.dt, pr.dt)
        assert abs(c[i] - xs) < 1e-13


def test_backtrack_time_only_speed_equals_fine_steps_2d(oracle):
    nx, m = 16, 4
    pr = _prob(2, nx, m, 1.3, 3, 3, [W.term(1.0, kt=2.0)], [W.term(-0.7, kt=1.0), W.term(0.2)])
    deps = [oracle.depart_fine(pr, k) for k in range(m)]
    cx, cy = oracle.backtrack_2d(nx, m, np.stack([d[0] for d in deps]), np.stack([d[1] for d in deps]))
    h = pr.h
    for idx in (0, 17, 100, 255):
        xs, ys = -1 + (idx % nx) * h, -1 + (idx // nx) * h
        for k in range(m - 1, -1, -1):
            xs, ys = oracle.erk_back(pr, xs, ys, (k + 1) * pr.dt, pr.dt)
        assert abs(cx[idx] - xs) < 1e-13 and abs(cy[idx] - ys) < 1e-13


def test_backtrack_periodic_wrap(oracle):
    """Shifting every sub-step's departure map by one period (2) shifts the
    composed coarse departure point by m periods: the periodic extension of
    the departure maps is consistent across the seam."""
    nx, m = 32, 4
    pr = _prob(1, nx, m, 3.7, 1, 1, W.alpha_cfg12())
    fine = np.stack([oracle.depart_fine(pr, k)[0] for k in range(m)])
    c0 = oracle.backtrack_1d(nx, m, fine)
    c1 = oracle.backtrack_1d(nx, m, fine + 2.0)
    assert np.abs(c1 - (c0 + 2.0 * m)).max() < 1e-12


# ------------------------------------------------------------ phi / sigma
@pytest.mark.parametrize("p,value", [(1, 0.135), (3, -0.022809375)])
def test_phi_worked_value_constant_speed(oracle, p, value):
    """Constant speed (Sec. 3.2): phi = f(frac(m c)) - m f(frac(c)), constant
    in space; c = 0.85, m = 4 gives 0.135 (p=1) and -0.022809375 (p=3)."""
    pr = _prob(1, 64, 64, 0.85, p, p, [W.term(1.0)])
    sv = W.Solver(m=[4], max_levels=3)
    ctx = oracle.Context(pr, sv)
    s1 = ctx.sigma(1)
    assert np.abs(s1 - value).max() < 1e-12
    # level 2: sigma = sum of the m level-1 sigmas + phi^(2), eq. (nu_p_def)
    f = oracle.fpoly
    phi2 = f(p, (16 * 0.85) % 1.0) - 4 * f(p, (4 * 0.85) % 1.0)
    assert np.abs(ctx.sigma(2) - (4 * value + phi2)).max() < 1e-12


def test_sigma_makes_B_dissipative(oracle):
    """Odd p: the backward-Euler factor has symbol 1/(1 - sigma*lambda_D) <= 1
    for constant speed, i.e. sigma*lambda_D <= 0 (Sec. 3.2)."""
    for p in (1, 3, 5):
        for cfl in (0.3, 0.85, 2.4, 4.0 + 1e-3):
            pr = _prob(1, 32, 64, cfl, p, p, [W.term(1.0)])
            ctx = oracle.Context(pr, W.Solver(m=[4], max_levels=2))
            s = ctx.sigma(1)[0, 0]
            lam = (-4.0) ** ((p + 1) // 2)   # symbol of D_{p+1} at omega = pi
            assert s * lam <= 1e-15, (p, cfl, s)


# ------------------------------------------------------------ GMRES
@pytest.mark.parametrize("dim,p", [(1, 1), (1, 3), (1, 5), (2, 3)])
def test_gmres_full_krylov_is_direct_solve(oracle, dim, p):
    nx = 8
    S = nx if dim == 1 else nx * nx
    rng = np.random.default_rng(2)
    sx = rng.uniform(0.0, 0.4, S) * (-1) ** ((p + 1) // 2 + 1)
    sy = rng.uniform(0.0, 0.4, S) * (-1) ** ((p + 1) // 2 + 1) if dim == 2 else None
    A = np.stack([oracle.apply_B(dim, nx, p, sx, sy, e) for e in np.eye(S)], axis=1)
    b = rng.standard_normal(S)
    y, it = oracle.bsolve(dim, nx, p, sx, sy, b, S, 0.0)
    assert np.abs(y - np.linalg.solve(A, b)).max() < 1e-10
    y0, it0 = oracle.bsolve(dim, nx, p, sx, sy, np.zeros(S), 10, 0.0)
    assert it0 == 0 and not y0.any()


def test_gmres_residual_nonincreasing_and_rtol_exit(oracle):
    nx, p = 64, 3
    rng = np.random.default_rng(3)
    sx = -rng.uniform(0.0, 0.5, nx)
    b = rng.standard_normal(nx)
    A = np.stack([oracle.apply_B(1, nx, p, sx, None, e) for e in np.eye(nx)], axis=1)
    prev = np.linalg.norm(b)
    for k in range(1, 11):
        y, it = oracle.bsolve(1, nx, p, sx, None, b, k, 0.0)
        assert it == k
        res = np.linalg.norm(b - A @ y)
        assert res <= prev * (1 + 1e-12)
        prev = res
    y, it = oracle.bsolve(1, nx, p, sx, None, b, 10, 1e-2)
    assert np.linalg.norm(b - A @ y) <= 1e-2 * np.linalg.norm(b) * (1 + 1e-9)
    if it > 1:
        y1, _ = oracle.bsolve(1, nx, p, sx, None, b, it - 1, 0.0)
        assert np.linalg.norm(b - A @ y1) > 1e-2 * np.linalg.norm(b)


# ------------------------------------------------------------ Lemma 3.3 / SM1
@pytest.mark.parametrize("p", [1, 3])
def test_modified_coarse_operator_truncation_order(oracle, p):
    """SM1 with alpha = cos(2 pi t), exact departure points: the quantity
    ||prod S_fine u - C S_coarse u||_inf / ||phi||_inf decays like h^{p+1} for
    C = I and like h^{p+2} for C = B_{p+1} (Lemma 3.3)."""
    m = 4
    res_I, res_B = [], []
    for nx in (64, 128, 256, 512):
        h = 2.0 / nx
        dt = 0.85 * h
        x = I.mesh(nx)
        shift = lambda t0, t1: (math.sin(2 * math.pi * t1) - math.sin(2 * math.pi * t0)) / (2 * math.pi)
        u = np.sin(math.pi * x) + 0.5 * np.cos(3 * math.pi * x + 0.2)
        v = u.copy()
        fs = 0.0
        for k in range(m):
            xi = x - shift(k * dt, (k + 1) * dt)
            v = oracle.interp(1, nx, p, xi, None, v)
            fs += oracle.fpoly(p, oracle.decompose(nx, xi[0])[1])
        xc = x - shift(0.0, m * dt)
        Sc = oracle.interp(1, nx, p, xc, None, u)
        phi = (-1) ** (p + 1) * (oracle.fpoly(p, oracle.decompose(nx, xc[0])[1]) - fs)
        sig = np.full(nx, phi)
        B = np.stack([oracle.apply_B(1, nx, p, sig, None, e) for e in np.eye(nx)], axis=1)
        BSc = np.linalg.solve(B, Sc)                   # the exact inverse of B
        res_I.append(np.abs(v - Sc).max() / abs(phi))
        res_B.append(np.abs(v - BSc).max() / abs(phi))
    oI = [math.log2(res_I[i] / res_I[i + 1]) for i in range(3)]
    oB = [math.log2(res_B[i] / res_B[i + 1]) for i in range(3)]
    assert np.mean(oI[1:]) > p + 1 - 0.3, oI
    assert np.mean(oB[1:]) > p + 2 - 0.3, oB


@pytest.mark.parametrize("dim,p,k", [(1, 1, 3), (1, 3, 5), (1, 5, 6), (2, 3, 4)])
def test_gmres_iterate_minimises_residual_over_krylov_space(oracle, dim, p, k):
    """After k iterations (rtol = 0) GMRES returns the minimiser of
    ||b - B y|| over the Krylov space span{b, Bb, ..., B^{k-1} b} (the
    definition of GMRES, Sec. 3.3), computed here by a least-squares solve
    on the explicit power basis."""
    nx = 12
    S = nx if dim == 1 else nx * nx
    rng = np.random.default_rng(5 + k)
    sgn = (-1) ** ((p + 1) // 2 + 1)
    sx = rng.uniform(0.0, 0.3, S) * sgn
    sy = rng.uniform(0.0, 0.3, S) * sgn if dim == 2 else None
    B = np.stack([oracle.apply_B(dim, nx, p, sx, sy, e) for e in np.eye(S)], axis=1)
    b = rng.standard_normal(S)
    K = [b]
    for _ in range(k - 1):
        K.append(B @ K[-1])
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    c, *_ = np.linalg.lstsq(B @ Q, b, rcond=None)
    y, it = oracle.bsolve(dim, nx, p, sx, sy, b, k, 0.0)
    assert it == k
    assert np.abs(y - Q @ c).max() < 1e-10 * np.abs(Q @ c).max()
