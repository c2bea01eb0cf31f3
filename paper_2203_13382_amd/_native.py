"""ctypes binding of ``libslmgrit.so`` (argument marshalling only).

Every step of the method runs in the HIP library; PyTorch provides device
memory and the stream.  Importing this module does not touch the GPU; the
library is loaded on first use and a missing library raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libslmgrit.so")

MAX_TERMS = 8
MAX_LEVELS = 24
SWEEP = {"FC": 0, "RES": 1, "F": 2}
STATUS = {0: "converged", 1: "not_converged", 2: "diverged", 3: "stagnated"}


class NativeError(RuntimeError):
    pass


class WaveTerm(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("coef", "kx", "px", "ky", "py", "kt", "pt")]


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("nt", C.c_int), ("dt", C.c_double),
                ("p", C.c_int), ("r", C.c_int),
                ("alpha", C.POINTER(WaveTerm)), ("n_alpha", C.c_int),
                ("beta", C.POINTER(WaveTerm)), ("n_beta", C.c_int),
                ("m", C.POINTER(C.c_int)), ("n_m", C.c_int),
                ("max_levels", C.c_int), ("coarsest_max_points", C.c_int),
                ("relax", C.c_int), ("gmres_kmax", C.c_int), ("gmres_rtol", C.c_double),
                ("tol", C.c_double), ("tol_mode", C.c_int), ("max_iter", C.c_int),
                ("precision", C.c_int), ("adjoint", C.c_int), ("coarse_op", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int), ("n_levels", C.c_int),
                ("rho0", C.c_double), ("rho_final", C.c_double), ("solve_ms", C.c_double),
                ("point_updates", C.c_longlong), ("gmres_solves", C.c_longlong),
                ("gmres_iters", C.c_longlong)]


# (name, restype, argtypes) for every function declared in include/slmgrit.h
_VP = C.c_void_p
SIGNATURES = [
    ("slm_plan_create", C.c_int, [C.POINTER(Desc), C.POINTER(_VP)]),
    ("slm_plan_destroy", None, [_VP]),
    ("slm_plan_workspace_size", C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    ("slm_plan_levels", C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int]),
    ("slm_plan_setup", C.c_int, [_VP, _VP, C.c_size_t, _VP]),
    ("slm_level_arrays", C.c_int, [_VP, C.c_int, C.POINTER(_VP), C.POINTER(C.c_int), C.POINTER(_VP)]),
    ("slm_autotune", C.c_int, [_VP, _VP, C.c_size_t, C.c_char_p, _VP]),
    ("slm_launch_info", C.c_int, [_VP, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("slm_apply_phi", C.c_int, [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP, _VP]),
    ("slm_relax", C.c_int, [_VP, C.c_int, C.c_int, _VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_double), _VP]),
    ("slm_relax_noalloc", C.c_int, [_VP, C.c_int, C.c_int, _VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_double), _VP]),
    ("slm_step", C.c_int, [_VP, _VP, _VP, C.c_int, _VP]),
    ("slm_seed_iterate", C.c_int, [_VP, C.c_uint64, _VP, C.c_int, _VP]),
    ("slm_solve", C.c_int, [_VP, _VP, _VP, C.POINTER(Stats), C.POINTER(C.c_double), C.c_int, _VP]),
    ("slm_solve_cpoints", C.c_int, [_VP, _VP, _VP, C.POINTER(Stats), C.POINTER(C.c_double), C.c_int, _VP]),
    ("slm_adjoint", C.c_int, [_VP, _VP, _VP, _VP, C.POINTER(C.c_double), C.POINTER(Stats),
                              C.POINTER(C.c_double), C.c_int, _VP]),
    ("slm_batch_create", C.c_int, [C.POINTER(Desc), C.c_int, C.POINTER(_VP)]),
    ("slm_batch_destroy", None, [_VP]),
    ("slm_batch_workspace_size", C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    ("slm_batch_setup", C.c_int, [_VP, _VP, C.c_size_t, _VP]),
    ("slm_batch_tune", C.c_int, [_VP, C.c_char_p, _VP]),
    ("slm_batch_solve", C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(Stats),
                                  C.POINTER(C.c_double), C.c_int, C.c_int, _VP]),
    ("slm_strerror", C.c_char_p, [C.c_int]),
    ("slm_last_error", C.c_char_p, [_VP]),
]

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise NativeError(f"{LIB} is missing: build it with paper_2203_13382_amd/build.py "
                              "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, plan=None, ok=(0,)):
    if rc in ok or rc > 0:
        return rc
    msg = lib().slm_last_error(plan).decode(errors="replace")
    raise NativeError(f"{lib().slm_strerror(rc).decode()} ({rc}): {msg}")


def terms_array(ts):
    arr = (WaveTerm * max(1, len(ts)))()
    for k, t in enumerate(ts):
        arr[k] = WaveTerm(*[float(v) for v in t])
    return arr


class _Keep:
    pass


def make_desc(pr, sv, precision: str, adjoint: bool = False):
    """Fill an ``slm_desc`` from a Problem/Solver pair; returns (desc, keepalive)."""
    keep = _Keep()
    keep.a = terms_array(pr.alpha)
    keep.b = terms_array(pr.beta or [])
    keep.m = (C.c_int * len(sv.m))(*sv.m)
    d = Desc(pr.dim, pr.nx, pr.nt, float(pr.dt), pr.p, pr.r, keep.a, len(pr.alpha),
             keep.b, len(pr.beta or []), keep.m, len(sv.m), sv.max_levels, sv.coarsest_max_points,
             {"F": 0, "FCF": 1}[sv.relax], sv.gmres_kmax, float(sv.gmres_rtol), float(sv.tol),
             {"abs": 0, "rel": 1}[sv.tol_mode], sv.max_iter, {"fp64": 0, "fp32": 1}[precision], int(bool(adjoint)),
             {"modified": 0, "ideal": 1, "redisc": 2, "fwd_euler": 3}[sv.coarse_op])
    return d, keep
