"""Pins of the oracle's scalar building blocks against closed forms.

Each test checks a fact fixed by the paper or by mathematics, not by the
oracle's own formulas: Runge-Kutta order conditions and observed orders,
polynomial reproduction of Lagrange interpolation, the interpolation error
polynomial f_{p+1} (eq. fpoly_def) and the symbol of D_{p+1} (eq. Dp+1_def).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2203_13382_amd import workloads as W


# ------------------------------------------------------------ ERK tableaux
def _order_conditions(r):
    """Butcher order conditions up to order r as (name, function of (c, A, b),
    exact value).  Written from the rooted-tree conditions, not from the
    oracle's code."""
    conds = [("b.1", lambda c, A, b: sum(b), Fraction(1))]
    if r >= 2:
        conds += [("b.c", lambda c, A, b: sum(bi * ci for bi, ci in zip(b, c)), Fraction(1, 2))]
    if r >= 3:
        conds += [("b.c2", lambda c, A, b: sum(bi * ci**2 for bi, ci in zip(b, c)), Fraction(1, 3)),
                  ("b.Ac", lambda c, A, b: sum(b[i] * sum(A[i][j] * c[j] for j in range(len(c)))
                                               for i in range(len(c))), Fraction(1, 6))]
    if r >= 4:
        def Ac(c, A):
            return [sum(A[i][j] * c[j] for j in range(len(c))) for i in range(len(c))]

        def Ac2(c, A):
            return [sum(A[i][j] * c[j] ** 2 for j in range(len(c))) for i in range(len(c))]

        def AAc(c, A):
            v = Ac(c, A)
            return [sum(A[i][j] * v[j] for j in range(len(c))) for i in range(len(c))]
        conds += [("b.c3", lambda c, A, b: sum(bi * ci**3 for bi, ci in zip(b, c)), Fraction(1, 4)),
                  ("b.cAc", lambda c, A, b: sum(b[i] * c[i] * Ac(c, A)[i] for i in range(len(c))), Fraction(1, 8)),
                  ("b.Ac2", lambda c, A, b: sum(b[i] * Ac2(c, A)[i] for i in range(len(c))), Fraction(1, 12)),
                  ("b.AAc", lambda c, A, b: sum(b[i] * AAc(c, A)[i] for i in range(len(c))), Fraction(1, 24))]
    if r >= 5:
        def mv(A, v):
            return [sum(A[i][j] * v[j] for j in range(len(v))) for i in range(len(v))]

        def cond(f, val):
            return (f.__name__, f, val)

        def t1(c, A, b): return sum(b[i] * c[i] ** 4 for i in range(len(c)))
        def t2(c, A, b): return sum(b[i] * c[i] ** 2 * mv(A, c)[i] for i in range(len(c)))
        def t3(c, A, b): return sum(b[i] * c[i] * mv(A, [x * x for x in c])[i] for i in range(len(c)))
        def t4(c, A, b): return sum(b[i] * c[i] * mv(A, mv(A, c))[i] for i in range(len(c)))
        def t5(c, A, b): return sum(b[i] * mv(A, c)[i] ** 2 for i in range(len(c)))
        def t6(c, A, b): return sum(b[i] * mv(A, [x ** 3 for x in c])[i] for i in range(len(c)))
        def t7(c, A, b): return sum(b[i] * mv(A, [c[j] * mv(A, c)[j] for j in range(len(c))])[i] for i in range(len(c)))
        def t8(c, A, b): return sum(b[i] * mv(A, mv(A, [x * x for x in c]))[i] for i in range(len(c)))
        def t9(c, A, b): return sum(b[i] * mv(A, mv(A, mv(A, c)))[i] for i in range(len(c)))
        conds += [cond(t1, Fraction(1, 5)), cond(t2, Fraction(1, 10)), cond(t3, Fraction(1, 15)),
                  cond(t4, Fraction(1, 30)), cond(t5, Fraction(1, 20)), cond(t6, Fraction(1, 20)),
                  cond(t7, Fraction(1, 40)), cond(t8, Fraction(1, 60)), cond(t9, Fraction(1, 120))]
    return conds


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5])
def test_erk_order_conditions(oracle, r):
    s, c, A, b = oracle.erk_tableau(r)
    assert s >= r
    # consistency: row sums of A equal c
    assert np.allclose(A.sum(axis=1), c, atol=1e-15)
    for name, f, val in _order_conditions(r):
        assert abs(f(list(c), [list(row) for row in A], list(b)) - float(val)) < 1e-14, (r, name)
    if r < 5:   # the next order fails (so the order is exactly r)
        higher = _order_conditions(r + 1)[len(_order_conditions(r)):]
        assert any(abs(f(list(c), [list(row) for row in A], list(b)) - float(v)) > 1e-6
                   for _, f, v in higher)


@pytest.mark.parametrize("r", [1, 3, 5])
def test_erk_observed_order(oracle, r):
    """Local error of one backward ERK step on a spatially varying alpha is
    O(dt^{r+1}) (Sec. 2.1); reference: 4000 classical RK4 substeps."""
    pr = W.Problem(1, 64, 1, 0.1, 1, r, W.alpha_cfg12())

    def alpha(x, t):
        return 1.0 + 0.5 * math.sin(math.pi * x) * math.cos(2 * math.pi * t)

    def ref(x, t_arr, dt, n=4000):
        hs = -dt / n
        t = t_arr
        for _ in range(n):
            k1 = alpha(x, t)
            k2 = alpha(x + hs / 2 * k1, t + hs / 2)
            k3 = alpha(x + hs / 2 * k2, t + hs / 2)
            k4 = alpha(x + hs * k3, t + hs)
            x += hs / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            t += hs
        return x

    errs = []
    dts = {1: [0.04, 0.02, 0.01], 3: [0.1, 0.05, 0.025], 5: [0.05, 0.025, 0.0125]}[r]
    for dt in dts:
        xd, _ = oracle.erk_back(pr, 0.3, 0.0, 0.7, dt)
        errs.append(abs(xd - ref(0.3, 0.7, dt)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > r + 1 - 0.5, (r, errs, orders)


def test_erk_exact_for_constant_speed(oracle):
    pr = W.Problem(1, 64, 1, 0.1, 1, 5, [W.term(0.75)])
    for r in (1, 3, 5):
        pr.r = r
        xd, _ = oracle.erk_back(pr, 0.25, 0.0, 1.0, 0.1)
        assert abs(xd - (0.25 - 0.075)) < 1e-15


def test_wave_terms(oracle):
    # sin(pi x) written as cos(pi x - pi/2); alpha of the 1D configs
    a = W.alpha_cfg12()
    for x, t in [(0.3, 0.1), (-0.7, 2.25), (0.0, 0.5)]:
        assert abs(oracle.wave(a, x, 0.0, t) - (1 + 0.5 * math.sin(math.pi * x) * math.cos(2 * math.pi * t))) < 1e-15


# ------------------------------------------------------------ interpolation
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_weights_reproduce_polynomials(oracle, p):
    """Degree-p Lagrange interpolation through x_E + jh is exact for
    polynomials of degree <= p: sum_j w_j j^q = (-eps)^q (Sec. 2.1)."""
    rng = np.random.default_rng(0)
    for eps in list(rng.random(20)) + [0.0, 0.5, 0.999999]:
        ell, rr = oracle.stencil(p, eps)
        assert ell + rr == p
        w = oracle.weights(p, eps)
        j = np.arange(-ell, rr + 1)
        for q in range(p + 1):
            assert abs(np.sum(w * j.astype(float) ** q) - (-eps) ** q) < 1e-13


def test_weights_linear_closed_form(oracle):
    for eps in (0.0, 0.25, 0.85):
        assert np.allclose(oracle.weights(1, eps), [eps, 1 - eps], atol=1e-16)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_stencil_is_nearest_nodes(oracle, p):
    """The p+1 nodes are the nearest neighbours of the departure point
    (Sec. 2.1): every node outside is at least as far as every node inside."""
    for eps in np.linspace(0.01, 0.99, 37):
        ell, rr = oracle.stencil(p, eps)
        inside = [abs(j + eps) for j in range(-ell, rr + 1)]
        outside = [abs(-ell - 1 + eps), abs(rr + 1 + eps)]
        assert max(inside) <= min(outside) + 1e-12


def test_fpoly_closed_values(oracle):
    assert oracle.fpoly(1, 0.5) == -1.0 / 8
    assert abs(oracle.fpoly(3, 0.5) - 3.0 / 128) < 1e-17
    assert abs(oracle.fpoly(5, 0.5) + 5.0 / 1024) < 1e-17
    for p in (1, 3, 5):
        assert oracle.fpoly(p, 0.0) == 0.0
        assert abs(oracle.fpoly(p, 1.0)) < 1e-16


@pytest.mark.parametrize("p", [1, 3, 5])
def test_fpoly_is_interpolation_error(oracle, p):
    """Eq. (poly_interp_error): interpolating x^{p+1} at x_E - h eps errs by
    exactly (-h)^{p+1} f_{p+1}(eps) (p+1)!."""
    h, xE = 0.125, 0.3
    for eps in (0.1, 0.37, 0.5, 0.81):
        ell, rr = oracle.stencil(p, eps)
        w = oracle.weights(p, eps)
        nodes = xE + h * np.arange(-ell, rr + 1)
        xi = xE - h * eps
        err = xi ** (p + 1) - np.sum(w * nodes ** (p + 1))
        assert abs(err - (-h) ** (p + 1) * oracle.fpoly(p, eps) * math.factorial(p + 1)) < 1e-13


def test_decompose(oracle):
    nx = 64
    h = 2.0 / nx
    E, eps = oracle.decompose(nx, -1.0 + 5 * h)        # on a node
    assert (E, eps) == (5, 0.0)
    E, eps = oracle.decompose(nx, -1.0 + 5.25 * h)
    assert E == 6 and abs(eps - 0.75) < 1e-12
    E, eps = oracle.decompose(nx, -1.0 - 2.5 * h)      # west of the domain: unwrapped
    assert E == -2 and abs(eps - 0.5) < 1e-12


# ------------------------------------------------------------ D_{p+1}
@pytest.mark.parametrize("p", [1, 3, 5])
def test_dop_symbol_and_order(oracle, p):
    """D_{p+1} is circulant; on a periodic grid sin(w x) is an eigenvector.
    h^{-(p+1)} D_{p+1} approximates the (p+1)-st derivative to second order
    (eq. Dp+1_def with s = 2) and annihilates constants."""
    q = (p + 1) // 2
    errs = []
    for nx in (32, 64, 128):
        h = 2.0 / nx
        x = -1.0 + h * np.arange(nx)
        v = np.sin(3 * math.pi * x)
        Dv = oracle.apply_D(nx, p, v)
        sym = (-4 * math.sin(3 * math.pi * h / 2) ** 2) ** q
        assert np.allclose(Dv, sym * v, atol=1e-12 * max(1, abs(sym)))
        exact = (-1) ** q * (3 * math.pi) ** (2 * q) * v
        errs.append(np.abs(Dv / h ** (p + 1) - exact).max())
        assert np.abs(oracle.apply_D(nx, p, np.ones(nx))).max() < 1e-12
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.9, orders
