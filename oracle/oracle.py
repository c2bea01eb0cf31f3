"""ctypes wrapper around the FP64 CPU oracle (``slmo.c``).

Test infrastructure only: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module; the GPU library
never does.  Problems and solver settings are passed as plain objects with
the attributes of ``slmo_problem`` / ``slmo_solver`` (see ``slmo.h``); this
module reads those attributes and nothing else of the package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "slmo.c")
LIB = os.path.join(HERE, "libslmo.so")

RELAX = {"F": 0, "FCF": 1}
COARSE = {"modified": 0, "ideal": 1, "redisc": 2, "fwd_euler": 3}
TOLMODE = {"abs": 0, "rel": 1}
STATUS = {0: "converged", 1: "not_converged", 2: "diverged"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libslmo.so``."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-fopenmp",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Term(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("coef", "kx", "px", "ky", "py", "kt", "pt")]


class CProblem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("nt", C.c_int), ("dt", C.c_double),
                ("p", C.c_int), ("r", C.c_int),
                ("alpha", C.POINTER(Term)), ("n_alpha", C.c_int),
                ("beta", C.POINTER(Term)), ("n_beta", C.c_int)]


class CSolver(C.Structure):
    _fields_ = [("m", C.POINTER(C.c_int)), ("n_m", C.c_int), ("max_levels", C.c_int),
                ("coarsest_max_points", C.c_int), ("relax", C.c_int), ("coarse_op", C.c_int),
                ("gmres_kmax", C.c_int), ("gmres_rtol", C.c_double), ("tol", C.c_double),
                ("tol_mode", C.c_int), ("max_iter", C.c_int)]


class CStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int), ("n_levels", C.c_int),
                ("rho0", C.c_double), ("rho_final", C.c_double),
                ("gmres_solves", C.c_longlong), ("gmres_iters", C.c_longlong)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        L.slmo_wave.restype = C.c_double
        L.slmo_wave.argtypes = [C.POINTER(Term), C.c_int, C.c_double, C.c_double, C.c_double]
        L.slmo_erk_tableau.argtypes = [C.c_int, _D, _D, _D]
        L.slmo_erk_back.argtypes = [C.POINTER(CProblem), C.c_double, C.c_double, C.c_double,
                                    C.c_double, _D, _D]
        L.slmo_stencil.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.slmo_weights.argtypes = [C.c_int, C.c_double, _D]
        L.slmo_fpoly.restype = C.c_double
        L.slmo_fpoly.argtypes = [C.c_int, C.c_double]
        L.slmo_dop_taps.argtypes = [C.c_int, _D]
        L.slmo_decompose.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_longlong), _D]
        L.slmo_depart_fine.argtypes = [C.POINTER(CProblem), C.c_int, _D, _D]
        L.slmo_interp.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, _D]
        L.slmo_apply_D.argtypes = [C.c_int, C.c_int, _D, _D]
        L.slmo_apply_B.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, _D]
        L.slmo_bsolve.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, _D, C.c_int, C.c_double]
        L.slmo_backtrack_1d.argtypes = [C.c_int, C.c_int, _D, _D]
        L.slmo_backtrack_2d.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D]
        L.slmo_seq_fine.argtypes = [C.POINTER(CProblem), _D, _D]
        L.slmo_hierarchy.argtypes = [C.c_int, C.POINTER(CSolver), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.c_int]
        L.slmo_setup.restype = C.c_void_p
        L.slmo_setup.argtypes = [C.POINTER(CProblem), C.POINTER(CSolver)]
        L.slmo_free.argtypes = [C.c_void_p]
        L.slmo_levels.argtypes = [C.c_void_p]
        L.slmo_level_N.argtypes = [C.c_void_p, C.c_int]
        L.slmo_level_m.argtypes = [C.c_void_p, C.c_int]
        L.slmo_level_dep.restype = _D
        L.slmo_level_dep.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.slmo_level_sigma.restype = _D
        L.slmo_level_sigma.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.slmo_apply_phi.argtypes = [C.c_void_p, C.c_int, C.c_int, _D, _D]
        L.slmo_mgrit.argtypes = [C.c_void_p, _D, _D, _D, C.c_int, C.POINTER(CStats)]
        L.slmo_apply_BT.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, _D]
        L.slmo_bsolve_T.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, _D, C.c_int, C.c_double]
        L.slmo_interp_T.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D, _D, _D]
        L.slmo_apply_phi_T.argtypes = [C.c_void_p, C.c_int, C.c_int, _D, _D]
        L.slmo_adjoint_seq.argtypes = [C.POINTER(CProblem), _D, _D]
        L.slmo_mgrit_adjoint.argtypes = [C.c_void_p, _D, _D, _D, C.c_int, C.POINTER(CStats)]
        L.slmo_erk_back_tangent.argtypes = [C.POINTER(CProblem), C.c_double, C.c_double, C.c_double,
                                            C.c_double, _D, _D]
        L.slmo_weights_deps.argtypes = [C.c_int, C.c_double, _D]
        L.slmo_grad_theta.argtypes = [C.POINTER(CProblem), _D, _D, _D]
        L.slmo_set_threads.argtypes = [C.c_int]
        L.slmo_get_threads.restype = C.c_int
        L.slmo_splitmix64.restype = C.c_uint64
        L.slmo_splitmix64.argtypes = [C.c_uint64]
        L.slmo_seeded_value.restype = C.c_double
        L.slmo_seeded_value.argtypes = [C.c_uint64, C.c_uint64]
        L.slmo_seeded_iterate.argtypes = [C.c_uint64, C.c_int, C.c_longlong, C.c_int, _D]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _terms(ts):
    arr = (Term * max(1, len(ts)))()
    for k, t in enumerate(ts):
        arr[k] = Term(*[float(v) for v in t])
    return arr


class _Keep:
    """Keeps the ctypes arrays a struct points into alive."""


def c_problem(pr):
    keep = _Keep()
    keep.a = _terms(pr.alpha)
    keep.b = _terms(getattr(pr, "beta", []) or [])
    cp = CProblem(pr.dim, pr.nx, pr.nt, float(pr.dt), pr.p, pr.r,
                  keep.a, len(pr.alpha), keep.b, len(getattr(pr, "beta", []) or []))
    keep.cp = cp
    return keep


def c_solver(sv):
    keep = _Keep()
    keep.m = (C.c_int * len(sv.m))(*sv.m)
    keep.cs = CSolver(keep.m, len(sv.m), sv.max_levels, sv.coarsest_max_points,
                      RELAX[sv.relax], COARSE[sv.coarse_op], sv.gmres_kmax,
                      float(sv.gmres_rtol), float(sv.tol), TOLMODE[sv.tol_mode], sv.max_iter)
    return keep


def S_of(pr):
    return pr.nx if pr.dim == 1 else pr.nx * pr.nx


# ---------------------------------------------------------------- scalar API
def erk_tableau(r):
    c = np.zeros(6); a = np.zeros(36); b = np.zeros(6)
    s = lib().slmo_erk_tableau(r, _ptr(c), _ptr(a), _ptr(b))
    return s, c[:s].copy(), a.reshape(6, 6)[:s, :s].copy(), b[:s].copy()


def wave(terms, x, y, t):
    arr = _terms(terms)
    return lib().slmo_wave(arr, len(terms), x, y, t)


def erk_back(pr, x, y, t_arr, dt):
    k = c_problem(pr)
    xd = C.c_double(); yd = C.c_double()
    lib().slmo_erk_back(C.byref(k.cp), x, y, t_arr, dt, C.byref(xd), C.byref(yd))
    return xd.value, yd.value


def stencil(p, eps):
    a = C.c_int(); b = C.c_int()
    lib().slmo_stencil(p, eps, C.byref(a), C.byref(b))
    return a.value, b.value


def weights(p, eps):
    w = np.zeros(p + 1)
    lib().slmo_weights(p, eps, _ptr(w))
    return w


def fpoly(p, z):
    return lib().slmo_fpoly(p, z)


def dop_taps(p):
    t = np.zeros(p + 2)
    lib().slmo_dop_taps(p, _ptr(t))
    return t


def decompose(nx, xi):
    E = C.c_longlong(); e = C.c_double()
    lib().slmo_decompose(nx, xi, C.byref(E), C.byref(e))
    return E.value, e.value


# ---------------------------------------------------------------- vector API
def depart_fine(pr, n):
    S = S_of(pr)
    xi = np.zeros(S); eta = np.zeros(S)
    k = c_problem(pr)
    lib().slmo_depart_fine(C.byref(k.cp), n, _ptr(xi), _ptr(eta))
    return (xi,) if pr.dim == 1 else (xi, eta)


def interp(dim, nx, p, xi, eta, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().slmo_interp(dim, nx, p, _ptr(np.ascontiguousarray(xi)),
                      _ptr(None if eta is None else np.ascontiguousarray(eta)), _ptr(u), _ptr(out))
    return out


def apply_D(nx, p, v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    lib().slmo_apply_D(nx, p, _ptr(v), _ptr(out))
    return out


def apply_B(dim, nx, p, sx, sy, v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    lib().slmo_apply_B(dim, nx, p, _ptr(np.ascontiguousarray(sx)),
                       _ptr(None if sy is None else np.ascontiguousarray(sy)), _ptr(v), _ptr(out))
    return out


def bsolve(dim, nx, p, sx, sy, b, kmax, rtol):
    b = np.ascontiguousarray(b, dtype=np.float64)
    y = np.zeros_like(b)
    it = lib().slmo_bsolve(dim, nx, p, _ptr(np.ascontiguousarray(sx)),
                           _ptr(None if sy is None else np.ascontiguousarray(sy)),
                           _ptr(b), _ptr(y), kmax, float(rtol))
    return y, it


def backtrack_1d(nx, m, fine):
    fine = np.ascontiguousarray(fine, dtype=np.float64)
    out = np.zeros(nx)
    lib().slmo_backtrack_1d(nx, m, _ptr(fine), _ptr(out))
    return out


def backtrack_2d(nx, m, fxi, feta):
    fxi = np.ascontiguousarray(fxi, dtype=np.float64)
    feta = np.ascontiguousarray(feta, dtype=np.float64)
    cx = np.zeros(nx * nx); cy = np.zeros(nx * nx)
    lib().slmo_backtrack_2d(nx, m, _ptr(fxi), _ptr(feta), _ptr(cx), _ptr(cy))
    return cx, cy


def seq_fine(pr, u0):
    S = S_of(pr)
    u = np.zeros((pr.nt + 1, S))
    k = c_problem(pr)
    lib().slmo_seq_fine(C.byref(k.cp), _ptr(np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)),
                        _ptr(u))
    return u


def apply_BT(dim, nx, p, sx, sy, v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    lib().slmo_apply_BT(dim, nx, p, _ptr(np.ascontiguousarray(sx)),
                        _ptr(None if sy is None else np.ascontiguousarray(sy)), _ptr(v), _ptr(out))
    return out


def bsolve_T(dim, nx, p, sx, sy, b, kmax, rtol):
    b = np.ascontiguousarray(b, dtype=np.float64)
    y = np.zeros_like(b)
    it = lib().slmo_bsolve_T(dim, nx, p, _ptr(np.ascontiguousarray(sx)),
                             _ptr(None if sy is None else np.ascontiguousarray(sy)),
                             _ptr(b), _ptr(y), kmax, float(rtol))
    return y, it


def interp_T(dim, nx, p, xi, eta, lam):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros_like(lam)
    lib().slmo_interp_T(dim, nx, p, _ptr(np.ascontiguousarray(xi)),
                        _ptr(None if eta is None else np.ascontiguousarray(eta)), _ptr(lam), _ptr(out))
    return out


def adjoint_seq(pr, lamT):
    """lambda_n for n = 0..nt from lambda_nt = lamT (sequential S_n^T sweep)."""
    S = S_of(pr)
    lam = np.zeros((pr.nt + 1, S))
    k = c_problem(pr)
    lib().slmo_adjoint_seq(C.byref(k.cp), _ptr(np.ascontiguousarray(lamT, dtype=np.float64).reshape(-1)),
                           _ptr(lam))
    return lam


def n_theta(pr):
    return len(pr.alpha) + (len(pr.beta or []) if pr.dim == 2 else 0)


def erk_back_tangent(pr, x, y, t_arr, dt):
    nq = n_theta(pr)
    dxi, deta = np.zeros(16), np.zeros(16)
    k = c_problem(pr)
    lib().slmo_erk_back_tangent(C.byref(k.cp), x, y, t_arr, dt, _ptr(dxi), _ptr(deta))
    return dxi[:nq].copy(), deta[:nq].copy()


def weights_deps(p, eps):
    w = np.zeros(p + 1)
    lib().slmo_weights_deps(p, eps, _ptr(w))
    return w


def grad_theta(pr, u_all, lam_all):
    g = np.zeros(16)
    k = c_problem(pr)
    lib().slmo_grad_theta(C.byref(k.cp), _ptr(np.ascontiguousarray(u_all, dtype=np.float64)),
                          _ptr(np.ascontiguousarray(lam_all, dtype=np.float64)), _ptr(g))
    return g[:n_theta(pr)].copy()


def loss_and_gradient(pr, u0, u_obs):
    """L = 1/2 ||u_nt - u_obs||^2 of sequential stepping, dL/du0 and dL/dtheta
    (theta = the alpha term coefficients, then the beta ones in 2D)."""
    u = seq_fine(pr, u0)
    r = u[-1] - np.asarray(u_obs, dtype=np.float64).reshape(-1)
    lam = adjoint_seq(pr, r)
    return 0.5 * float(r @ r), lam[0].copy(), grad_theta(pr, u, lam)


def set_threads(n):
    """Threads the oracle may use (OpenMP); results do not depend on it."""
    lib().slmo_set_threads(int(n))


def get_threads():
    return lib().slmo_get_threads()


def splitmix64(state):
    return lib().slmo_splitmix64(state & 0xFFFFFFFFFFFFFFFF)


def seeded_value(seed, idx):
    return lib().slmo_seeded_value(seed & 0xFFFFFFFFFFFFFFFF, idx & 0xFFFFFFFFFFFFFFFF)


def seeded_iterate(seed, nt, S, m0):
    """[(nt+1), S] array whose C-points (every m0-th time point) hold the
    seeded initial iterate (slmo_seeded_iterate); the rest is zero."""
    u = np.zeros((nt + 1, S))
    lib().slmo_seeded_iterate(seed & 0xFFFFFFFFFFFFFFFF, nt, S, m0, _ptr(u))
    return u


def hierarchy(nt, sv):
    N = (C.c_int * 64)(); mm = (C.c_int * 64)()
    k = c_solver(sv)
    L = lib().slmo_hierarchy(nt, C.byref(k.cs), N, mm, 64)
    return [N[i] for i in range(L)], [mm[i] for i in range(L)]


class Context:
    """Oracle setup (departure points and sigma on every level) + MGRIT."""

    def __init__(self, pr, sv):
        self.pr, self.sv = pr, sv
        self._kp, self._ks = c_problem(pr), c_solver(sv)
        self.h = lib().slmo_setup(C.byref(self._kp.cp), C.byref(self._ks.cs))
        self.S = S_of(pr)
        self.L = lib().slmo_levels(self.h)
        self.N = [lib().slmo_level_N(self.h, l) for l in range(self.L)]
        self.m = [lib().slmo_level_m(self.h, l) for l in range(self.L)]

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().slmo_free(self.h)
                self.h = None
        except Exception:
            pass

    def dep(self, level, comp=0):
        ptr = lib().slmo_level_dep(self.h, level, comp)
        n = self.N[level] * self.S
        return np.ctypeslib.as_array(ptr, shape=(n,)).reshape(self.N[level], self.S).copy()

    def sigma(self, level, comp=0):
        ptr = lib().slmo_level_sigma(self.h, level, comp)
        n = self.N[level] * self.S
        return np.ctypeslib.as_array(ptr, shape=(n,)).reshape(self.N[level], self.S).copy()

    def apply_phi(self, level, n, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        out = np.zeros_like(v)
        lib().slmo_apply_phi(self.h, level, n, _ptr(v), _ptr(out))
        return out

    def mgrit(self, u0, u_init, hist_cap=1000):
        """Run MGRIT.  ``u_init`` is [(nt+1), S]; its C-points are the initial
        iterate.  Returns (u, stats dict, residual history)."""
        u = np.ascontiguousarray(u_init, dtype=np.float64).reshape(self.pr.nt + 1, self.S).copy()
        hist = np.zeros(hist_cap)
        st = CStats()
        lib().slmo_mgrit(self.h, _ptr(np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)),
                         _ptr(u), _ptr(hist), hist_cap, C.byref(st))
        stats = dict(iterations=st.iterations, status=STATUS[st.status], n_levels=st.n_levels,
                     rho0=st.rho0, rho_final=st.rho_final, gmres_solves=st.gmres_solves,
                     gmres_iters=st.gmres_iters)
        nh = min(hist_cap, st.iterations) if st.n_levels > 1 else 0
        return u, stats, hist[:nh].copy()

    def apply_phi_T(self, level, n, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        out = np.zeros_like(v)
        lib().slmo_apply_phi_T(self.h, level, n, _ptr(v), _ptr(out))
        return out

    def mgrit_adjoint(self, lamT, mu_init, hist_cap=1000):
        """MGRIT on the adjoint system in reverse time: returns (mu, stats,
        history) with mu[k] = lambda_{nt-k}; ``mu_init``'s C-points are the
        initial iterate."""
        mu = np.ascontiguousarray(mu_init, dtype=np.float64).reshape(self.pr.nt + 1, self.S).copy()
        hist = np.zeros(hist_cap)
        st = CStats()
        lib().slmo_mgrit_adjoint(self.h, _ptr(np.ascontiguousarray(lamT, dtype=np.float64).reshape(-1)),
                                 _ptr(mu), _ptr(hist), hist_cap, C.byref(st))
        stats = dict(iterations=st.iterations, status=STATUS[st.status], n_levels=st.n_levels,
                     rho0=st.rho0, rho_final=st.rho_final, gmres_solves=st.gmres_solves,
                     gmres_iters=st.gmres_iters)
        nh = min(hist_cap, st.iterations) if st.n_levels > 1 else 0
        return mu, stats, hist[:nh].copy()
