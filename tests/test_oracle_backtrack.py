"""Pins of the oracle's backtracking of coarse departure points (Sec. 3.3.1,
eq. coarse_depart_interp; the bilinear 2D form of the supplement, eqs.
poly_interp_1d / poly_interp_2d) with departure maps that are not shifts.

With a space-independent speed every sub-step's departure map is a pure
shift, and then any node choice, either slope sign and either recursion
order give the same composed point.  These pins use maps for which those
choices matter:

* affine maps f_k(x) = a_k x + b_k (1D) and bilinear maps (2D) with
  step-dependent, non-commuting coefficients: linear (bilinear)
  interpolation reproduces them, so the backtracked point is the exact
  composition f_0(f_1(...f_{m-1}(x_i))) (arrival nodes away from the seam);
* periodic maps given only at the nodes (a random displacement per node and
  sub-step, several cells long, crossing the seam): the recursion is then the
  composition of the maps' piecewise-linear interpolants, evaluated here with
  numpy.interp (1D) and scipy's RegularGridInterpolator (2D);
* a smooth space-dependent speed: the backtracked point converges to m fine
  ERK steps at O(h^2) for a fixed step size (linear interpolation of a
  departure map whose curvature is O(dt)).

Each pin is shown to discriminate: the same checks are run on copies of the
oracle compiled with one planted mistake (slope sign, anchor node, cell
choice, recursion order, dropped periodic shift) and must fail there.
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

from paper_2203_13382_amd import inputs as I
from paper_2203_13382_amd import workloads as W

_D = C.POINTER(C.c_double)


def _bind(lib):
    lib.slmo_backtrack_1d.argtypes = [C.c_int, C.c_int, _D, _D]
    lib.slmo_backtrack_2d.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D]
    return lib


def _bt1(lib, nx, m, fine):
    fine = np.ascontiguousarray(fine, dtype=np.float64)
    out = np.zeros(nx)
    lib.slmo_backtrack_1d(nx, m, fine.ctypes.data_as(_D), out.ctypes.data_as(_D))
    return out


def _bt2(lib, nx, m, fx, fy):
    fx = np.ascontiguousarray(fx, dtype=np.float64)
    fy = np.ascontiguousarray(fy, dtype=np.float64)
    cx, cy = np.zeros(nx * nx), np.zeros(nx * nx)
    lib.slmo_backtrack_2d(nx, m, fx.ctypes.data_as(_D), fy.ctypes.data_as(_D),
                          cx.ctypes.data_as(_D), cy.ctypes.data_as(_D))
    return cx, cy


# ------------------------------------------------------------ the checks
def _affine_1d_error(bt, m=6, nx=128):
    """Max deviation from the exact composition of affine maps, over arrival
    nodes whose composed characteristic stays inside (-1, 1 - h)."""
    h = 2.0 / nx
    x = I.mesh(nx)
    rng = np.random.default_rng(11)
    a = 1.0 + rng.uniform(-0.12, 0.12, m)           # non-commuting: a_k and b_k vary with k
    b = rng.uniform(-0.08, 0.08, m)
    fine = np.stack([a[k] * x + b[k] for k in range(m)])
    c = bt(nx, m, fine)
    exact = x.copy()
    for k in range(m - 1, -1, -1):
        exact = a[k] * exact + b[k]
    inner = np.abs(x) < 0.45
    return np.abs(c - exact)[inner].max()


def _periodic_1d_error(bt, m=5, nx=64):
    """Departure maps given at the nodes only, f_k(x_i) = x_i - g_k[i] with
    a random displacement g of 1-6 cells (the characteristics cross the
    seam); reference: composition of the maps' piecewise-linear periodic
    interpolants (numpy.interp on the displacement, period 2)."""
    h = 2.0 / nx
    x = I.mesh(nx)
    rng = np.random.default_rng(12)
    g = rng.uniform(1.0, 6.0, (m, nx)) * h * np.where(rng.random(m) < 0.5, -1.0, 1.0)[:, None]
    fine = x[None, :] - g
    c = bt(nx, m, fine)
    ref = fine[m - 1].copy()
    for k in range(m - 2, -1, -1):
        ref = ref - np.interp(ref, x, g[k], period=2.0)
    return np.abs(c - ref).max()


def _bilinear_2d_error(bt, m=5, nx=48):
    """Bilinear maps X_k = a0 + a1 x + a2 y + a3 x y (Y_k likewise) with
    step-dependent coefficients: bilinear interpolation reproduces them, so
    the backtracked point is the exact composition."""
    h = 2.0 / nx
    x = I.mesh(nx)
    Xg, Yg = np.meshgrid(x, x, indexing="xy")
    X, Y = Xg.reshape(-1), Yg.reshape(-1)
    rng = np.random.default_rng(13)
    A = np.stack([rng.uniform(-0.06, 0.06, m), 1 + rng.uniform(-0.1, 0.1, m),
                  rng.uniform(-0.1, 0.1, m), rng.uniform(-0.1, 0.1, m)], 1)
    B = np.stack([rng.uniform(-0.06, 0.06, m), rng.uniform(-0.1, 0.1, m),
                  1 + rng.uniform(-0.1, 0.1, m), rng.uniform(-0.1, 0.1, m)], 1)
    fx = np.stack([A[k, 0] + A[k, 1] * X + A[k, 2] * Y + A[k, 3] * X * Y for k in range(m)])
    fy = np.stack([B[k, 0] + B[k, 1] * X + B[k, 2] * Y + B[k, 3] * X * Y for k in range(m)])
    cx, cy = bt(nx, m, fx, fy)
    ex, ey = X.copy(), Y.copy()
    for k in range(m - 1, -1, -1):
        ex, ey = (A[k, 0] + A[k, 1] * ex + A[k, 2] * ey + A[k, 3] * ex * ey,
                  B[k, 0] + B[k, 1] * ex + B[k, 2] * ey + B[k, 3] * ex * ey)
    inner = (np.abs(X) < 0.4) & (np.abs(Y) < 0.4)
    return max(np.abs(cx - ex)[inner].max(), np.abs(cy - ey)[inner].max())


def _periodic_2d_error(bt, m=4, nx=24):
    """Random periodic displacement fields per sub-step (1-4 cells in each
    component, crossing the seams); reference: composition of their bilinear
    interpolants (scipy RegularGridInterpolator on the grid extended by one
    periodic row and column)."""
    from scipy.interpolate import RegularGridInterpolator
    h = 2.0 / nx
    x = I.mesh(nx)
    Xg, Yg = np.meshgrid(x, x, indexing="xy")
    X, Y = Xg.reshape(-1), Yg.reshape(-1)
    rng = np.random.default_rng(14)
    gx = rng.uniform(1.0, 4.0, (m, nx, nx)) * h * np.where(rng.random(m) < 0.5, -1.0, 1.0)[:, None, None]
    gy = rng.uniform(1.0, 4.0, (m, nx, nx)) * h * np.where(rng.random(m) < 0.5, -1.0, 1.0)[:, None, None]
    fx = X[None, :] - gx.reshape(m, -1)
    fy = Y[None, :] - gy.reshape(m, -1)
    cx, cy = bt(nx, m, fx, fy)
    xe = np.append(x, 1.0)                         # grid of [-1, 1] with the periodic copy

    def ext(a):                                    # a[j, i] (y, x) -> periodic extension
        return np.pad(a, ((0, 1), (0, 1)), mode="wrap")

    rx, ry = fx[m - 1].copy(), fy[m - 1].copy()
    for k in range(m - 2, -1, -1):
        ix = RegularGridInterpolator((xe, xe), ext(gx[k]), method="linear")
        iy = RegularGridInterpolator((xe, xe), ext(gy[k]), method="linear")
        q = np.stack([np.mod(ry + 1.0, 2.0) - 1.0, np.mod(rx + 1.0, 2.0) - 1.0], 1)
        rx, ry = rx - ix(q), ry - iy(q)
    return max(np.abs(cx - rx).max(), np.abs(cy - ry).max())


def _checks_1d(lib):
    bt = lambda nx, m, f: _bt1(lib, nx, m, f)
    return {"affine": _affine_1d_error(bt), "periodic": _periodic_1d_error(bt)}


def _checks_2d(lib):
    bt = lambda nx, m, fx, fy: _bt2(lib, nx, m, fx, fy)
    return {"bilinear": _bilinear_2d_error(bt), "periodic": _periodic_2d_error(bt)}


# ------------------------------------------------------------ the oracle itself
def test_backtrack_1d_affine_maps_compose_exactly(oracle):
    assert _affine_1d_error(oracle.backtrack_1d) < 1e-13


def test_backtrack_1d_periodic_node_maps(oracle):
    assert _periodic_1d_error(oracle.backtrack_1d) < 1e-13


def test_backtrack_2d_bilinear_maps_compose_exactly(oracle):
    assert _bilinear_2d_error(oracle.backtrack_2d) < 1e-13


def test_backtrack_2d_periodic_node_maps(oracle):
    assert _periodic_2d_error(oracle.backtrack_2d) < 1e-13


def test_backtrack_1d_converges_to_fine_steps_at_second_order(oracle):
    """alpha = 1 + 0.5 sin(pi x) cos(2 pi t), fixed dt, m = 4: the
    backtracked coarse departure point against the characteristic traced
    through the m fine ERK steps (the exact composition of the fine maps)
    has an O(h^2) error (linear interpolation of maps with O(dt) curvature)."""
    m, dt = 4, 0.85 * 2.0 / 64
    errs = []
    for nx in (64, 128, 256, 512):
        pr = W.Problem(1, nx, m, dt, 3, 3, W.alpha_cfg12())
        fine = np.stack([oracle.depart_fine(pr, k)[0] for k in range(m)])
        c = oracle.backtrack_1d(nx, m, fine)
        x = I.mesh(nx)
        err = 0.0
        for i in range(nx):
            xs = x[i]
            for k in range(m - 1, -1, -1):
                xs, _ = oracle.erk_back(pr, xs, 0.0, (k + 1) * dt, dt)
            err = max(err, abs(c[i] - xs))
        errs.append(err)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    fit = -np.polyfit(np.log2([64, 128, 256, 512]), np.log2(errs), 1)[0]
    assert errs[0] > 1e-7, errs                    # the space dependence is felt
    assert fit > 1.85 and min(orders) > 1.6, (errs, orders, fit)


def test_backtrack_2d_converges_to_fine_steps_at_second_order(oracle):
    """The 2D field of the 512^2 workload, (cos(pi y) cos(pi t), sin(pi x)):
    the bilinear backtracking is O(h^2) close to the m fine ERK steps."""
    m, dt = 4, 2.0 * 2.0 / 32
    a, b = W.field_cfg3()
    errs = []
    for nx in (32, 64, 128):
        pr = W.Problem(2, nx, m, dt, 3, 3, a, b)
        deps = [oracle.depart_fine(pr, k) for k in range(m)]
        cx, cy = oracle.backtrack_2d(nx, m, np.stack([d[0] for d in deps]), np.stack([d[1] for d in deps]))
        h = 2.0 / nx
        err = 0.0
        for idx in range(0, nx * nx, max(1, nx * nx // 300) + 1):
            xs, ys = -1 + (idx % nx) * h, -1 + (idx // nx) * h
            for k in range(m - 1, -1, -1):
                xs, ys = oracle.erk_back(pr, xs, ys, (k + 1) * dt, dt)
            err = max(err, abs(cx[idx] - xs), abs(cy[idx] - ys))
        errs.append(err)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[0] > 1e-6, errs
    assert min(orders) > 1.8, (errs, orders)


# ------------------------------------------------------------ planted mistakes
_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "slmo.c")

# (name, [(text in slmo.c, replacement)], dimension)
_MUTANTS = [
    ("1d-slope-sign", [("c = (fE - fW) / h * (c - xE) + fE;", "c = (fW - fE) / h * (c - xE) + fE;")], 1),
    ("1d-anchor-west", [("c = (fE - fW) / h * (c - xE) + fE;", "c = (fE - fW) / h * (c - xE) + fW;")], 1),
    ("1d-cell-east", [("long long E = (long long)ceil((c + 1.0) / h), W = E - 1;\n            long long e = pmod(E, nx)",
                       "long long E = (long long)ceil((c + 1.0) / h) + 1, W = E - 1;\n            long long e = pmod(E, nx)")], 1),
    ("1d-forward-order", [("double c = fine[(long long)(m - 1) * nx + i];\n        for (int k = m - 2; k >= 0; k--)",
                           "double c = fine[(long long)(m - 1) * nx + i];\n        for (int k = 0; k <= m - 2; k++)")], 1),
    ("1d-no-period-shift", [("double fE = fine[(long long)k * nx + e] + (double)(E - e) * h;",
                             "double fE = fine[(long long)k * nx + e];")], 1),
    ("2d-slope-sign", [("return (qE - qW) / h * (x - xE) + qE;", "return (qW - qE) / h * (x - xE) + qE;")], 2),
    ("2d-north-south", [("return (north - south) / h * (y - yN) + north;",
                         "return (north - south) / h * (y - yN) + south;")], 2),
    ("2d-forward-order", [("double cy = feta[(long long)(m - 1) * S + id];\n        for (int k = m - 2; k >= 0; k--)",
                           "double cy = feta[(long long)(m - 1) * S + id];\n        for (int k = 0; k <= m - 2; k++)")], 2),
    ("2d-y-shift-from-north", [("Y[s * nx + e] + syS, Y[s * nx + w] + syS", "Y[s * nx + e] + syN, Y[s * nx + w] + syN")], 2),
    ("2d-components-swapped", [("cx = nx_; cy = ny_;", "cx = ny_; cy = nx_;")], 2),
]


def _build_mutant(tmp_path, name, subs):
    text = open(_SRC).read()
    for old, new in subs:
        assert text.count(old) == 1, (name, old)
        text = text.replace(old, new)
    src = tmp_path / f"slmo_{name}.c"
    src.write_text(text)
    so = tmp_path / f"libslmo_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I", os.path.dirname(_SRC),
                           "-o", str(so), str(src), "-lm"])
    return _bind(C.CDLL(str(so)))


@pytest.mark.parametrize("name,subs,dim", _MUTANTS, ids=[m[0] for m in _MUTANTS])
def test_planted_mistakes_fail_the_pins(tmp_path, name, subs, dim):
    """A copy of the oracle with one planted mistake must fail at least one
    of the pins above (each would pass a time-only-speed pin)."""
    lib = _build_mutant(tmp_path, name, subs)
    errs = _checks_1d(lib) if dim == 1 else _checks_2d(lib)
    assert max(errs.values()) > 1e-6, (name, errs)


def test_unmodified_copy_passes(tmp_path, oracle):
    """Control for the mutant harness: the copy built the same way without a
    change passes every pin."""
    lib = _build_mutant(tmp_path, "control", [])
    assert max(_checks_1d(lib).values()) < 1e-13
    assert max(_checks_2d(lib).values()) < 1e-13
