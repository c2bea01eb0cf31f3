"""Problem and solver descriptions for periodic linear advection with
semi-Lagrangian MGRIT (arXiv 2203.13382).

Plain data only: no arithmetic of the method lives here.  A wave speed is a
list of terms ``(coef, kx, px, ky, py, kt, pt)``, each meaning
``coef*cos(kx*pi*x+px)*cos(ky*pi*y+py)*cos(kt*pi*t+pt)``; the domain is
[-1,1)^dim with ``h = 2/nx``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

Term = Tuple[float, float, float, float, float, float, float]
HALF_PI = 0.5 * math.pi


@dataclass
class Problem:
    dim: int
    nx: int
    nt: int
    dt: float
    p: int
    r: int
    alpha: List[Term]
    beta: List[Term] = field(default_factory=list)

    @property
    def h(self) -> float:
        return 2.0 / self.nx

    @property
    def S(self) -> int:
        return self.nx if self.dim == 1 else self.nx * self.nx


@dataclass
class Solver:
    m: List[int]
    max_levels: int = 64
    coarsest_max_points: int = 2
    relax: str = "FCF"            # "F" or "FCF"
    coarse_op: str = "modified"   # "modified", "ideal", "redisc", "fwd_euler"
    gmres_kmax: int = 10
    gmres_rtol: float = 1e-2      # 0 => exactly gmres_kmax iterations
    tol: float = 1e-10
    tol_mode: str = "rel"         # "rel" or "abs"
    max_iter: int = 100


def term(coef, kx=0.0, px=0.0, ky=0.0, py=0.0, kt=0.0, pt=0.0) -> Term:
    return (float(coef), float(kx), float(px), float(ky), float(py), float(kt), float(pt))


def alpha_cfg12(amp: float = 0.5) -> List[Term]:
    """alpha(x,t) = 1 + amp*sin(pi x)*cos(2 pi t)."""
    return [term(1.0), term(amp, kx=1.0, px=-HALF_PI, kt=2.0)]


def field_cfg3() -> Tuple[List[Term], List[Term]]:
    """(alpha, beta) = (cos(pi y)*cos(pi t), sin(pi x))."""
    return [term(1.0, ky=1.0, kt=1.0)], [term(1.0, kx=1.0, px=-HALF_PI)]


def field_cfg5(theta=(1.0, 0.0, 1.0, 0.0)) -> Tuple[List[Term], List[Term]]:
    """alpha = th1*cos(pi y)cos(pi t) + th2*sin(2 pi y);
    beta = th3*sin(pi x) + th4*cos(2 pi x)cos(pi t)."""
    t1, t2, t3, t4 = theta
    return ([term(t1, ky=1.0, kt=1.0), term(t2, ky=2.0, py=-HALF_PI)],
            [term(t3, kx=1.0, px=-HALF_PI), term(t4, kx=2.0, kt=1.0)])


def config(n: int, **over):
    """The five benchmark workloads.  Returns (Problem, Solver, precision)."""
    if n == 1:
        nx = 64
        pr = Problem(1, nx, 256, 0.85 * 2.0 / nx, 1, 1, alpha_cfg12())
        sv = Solver(m=[4], max_levels=2, coarsest_max_points=2, relax="FCF",
                    gmres_kmax=10, gmres_rtol=0.0, tol=1e-10, tol_mode="abs", max_iter=100)
        prec = "fp64"
    elif n == 2:
        nx = 4096
        pr = Problem(1, nx, 16384, 4.0 * 2.0 / nx, 3, 3, alpha_cfg12())
        sv = Solver(m=[8], coarsest_max_points=16, relax="FCF", gmres_kmax=10,
                    gmres_rtol=1e-2, tol=1e-10, tol_mode="rel", max_iter=100)
        prec = "fp64"
    elif n == 3:
        nx = 512
        a, b = field_cfg3()
        pr = Problem(2, nx, 4096, 2.0 * 2.0 / nx, 5, 5, a, b)
        sv = Solver(m=[8], coarsest_max_points=16, relax="FCF", gmres_kmax=10,
                    gmres_rtol=1e-2, tol=1e-6, tol_mode="rel", max_iter=100)
        prec = "fp32"
    elif n == 5:
        nx = 256
        a, b = field_cfg5()
        pr = Problem(2, nx, 2048, 2.0 * 2.0 / nx, 3, 3, a, b)
        sv = Solver(m=[4], coarsest_max_points=16, relax="FCF", gmres_kmax=10,
                    gmres_rtol=1e-2, tol=1e-10, tol_mode="rel", max_iter=100)
        prec = "fp64"
    else:
        raise ValueError("config 4 is a batch: use batch_config()")
    pk = {k: v for k, v in over.items() if hasattr(pr, k)}
    sk = {k: v for k, v in over.items() if hasattr(sv, k)}
    pr = replace(pr, **pk)
    sv = replace(sv, **sk)
    if "dt_cfl" in over:
        pr = replace(pr, dt=over["dt_cfl"] * 2.0 / pr.nx)
    return pr, sv, over.get("precision", prec)


def scaled(pr: Problem, nx: int, nt: int, cfl: float) -> Problem:
    """Same PDE on another mesh with dt = cfl*h."""
    return replace(pr, nx=nx, nt=nt, dt=cfl * 2.0 / nx)


def batch_config(n: int = 64, seed: int = 4, cfl: float = 0.85, precision: str = "fp32", **over):
    """The batch workload: ``n`` independent 1D problems of the PDE of
    ``alpha_cfg12`` with drawn (nx, nt, p, amplitude) and dt = cfl*h, each
    with the multilevel solver of the 1D workload (m = 8 down to <= 16
    coarse points, FCF).  FP32 bulk stops at a relative tolerance of 1e-6
    (the FP32 floor; FP64 keeps 1e-10).  Returns (list of (Problem,
    Solver), precision)."""
    from .inputs import batch_draws
    tol = 1e-6 if precision == "fp32" else 1e-10
    out = []
    for d in batch_draws(n, seed):
        pr = Problem(1, d["nx"], d["nt"], cfl * 2.0 / d["nx"], d["p"], d["p"], alpha_cfg12(d["amp"]))
        sv = Solver(m=[8], coarsest_max_points=16, relax="FCF", gmres_kmax=10, gmres_rtol=1e-2,
                    tol=tol, tol_mode="rel", max_iter=100)
        pk = {k: v for k, v in over.items() if hasattr(pr, k)}
        sk = {k: v for k, v in over.items() if hasattr(sv, k)}
        out.append((replace(pr, **pk), replace(sv, **sk)))
    return out, precision


def adjoint_config(seed: int = 5, **over):
    """The adjoint workload: 2D, nx = ny = 256, nt = 2048, dt = 2h, p = r = 3,
    m = 4 down to <= 16 points, FCF, FP64, field_cfg5(theta).  The misfit
    target comes from theta_true = (1, 0, 1, 0) + 0.05 N(0,1); the gradient
    is taken at theta = (1, 0, 1, 0) + 0.02 N(0,1) (generic coefficients:
    at exactly (1, 0, 1, 0) some departure points sit on mesh nodes, where
    the interpolant's slope jumps).  Returns (Problem at theta, Solver,
    theta, theta_true)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    base = np.array([1.0, 0.0, 1.0, 0.0])
    theta_true = base + 0.05 * rng.standard_normal(4)
    theta = base + 0.02 * rng.standard_normal(4)
    nx = over.get("nx", 256)
    nt = over.get("nt", 2048)
    a, b = field_cfg5(tuple(theta))
    pr = Problem(2, nx, nt, 2.0 * 2.0 / nx, 3, 3, a, b)
    sv = Solver(m=[4], coarsest_max_points=16, relax="FCF", gmres_kmax=10, gmres_rtol=1e-2,
                tol=over.get("tol", 1e-10), tol_mode="rel", max_iter=100)
    return pr, sv, theta, theta_true


def paper_problem(dim: int, field: str, p: int, nx: int, nt: int) -> Problem:
    """The paper's test problems (Sec. 5 for 1D, Sec. 6 for 2D), dt = 0.85 h,
    r = p.  1D fields: 'a1' alpha = 1, 'a2' alpha = cos(2 pi t), 'a4' alpha =
    cos(2 pi t) cos(2 pi x); 2D: 'const' (alpha, beta) = (1, 1) and 'var', the
    time-dependent field of eq. (alpha-var_2D)."""
    dt = 0.85 * 2.0 / nx
    if dim == 2:
        kt = 2.0 / 3.4
        fields = {"const": ([term(1.0)], [term(1.0)]),
                  "var": ([term(0.5, kt=kt), term(-0.5, ky=2.0, kt=kt)],
                          [term(-0.5, kt=kt), term(-0.5, kx=2.0, kt=kt)])}
        a, b = fields[field]
        return Problem(2, nx, nt, dt, p, p, a, b)
    alpha = {"a1": [term(1.0)], "a2": [term(1.0, kt=2.0)], "a4": [term(1.0, kx=2.0, kt=2.0)]}[field]
    return Problem(1, nx, nt, dt, p, p, alpha, [])


def paper_initial_condition(dim: int, nx: int):
    """u0 = sin^4(pi x) in 1D; sin^2(pi/2 (x-1)) sin^2(pi/2 (y-1)) in 2D."""
    import numpy as np
    x = -1.0 + np.arange(nx) * (2.0 / nx)
    if dim == 1:
        return np.sin(np.pi * x) ** 4
    X, Y = np.meshgrid(x, x, indexing="xy")
    return (np.sin(np.pi / 2 * (X - 1)) ** 2 * np.sin(np.pi / 2 * (Y - 1)) ** 2).reshape(-1)

