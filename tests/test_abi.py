"""Host-only checks of the C ABI (no GPU needed): the library loads and
exports every function declared in include/slmgrit.h, descriptors are
validated, and the level hierarchy agrees with the oracle's."""
import ctypes as C
import os
import re

import pytest

from paper_2203_13382_amd import _native as N
from paper_2203_13382_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slmgrit.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(slm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert {n for n, _, _ in N.SIGNATURES} == set(names)


def _create(pr, sv, prec="fp64"):
    d, keep = N.make_desc(pr, sv, prec)
    h = C.c_void_p()
    rc = N.lib().slm_plan_create(C.byref(d), C.byref(h))
    return rc, h, keep


def _levels(h):
    nl = C.c_int()
    Ns = (C.c_int * 24)()
    ms = (C.c_int * 24)()
    assert N.lib().slm_plan_levels(h, C.byref(nl), Ns, ms, 24) == 0
    return [Ns[i] for i in range(nl.value)], [ms[i] for i in range(nl.value)]


@pytest.mark.parametrize("nt,kw", [
    (16384, dict(m=[8], coarsest_max_points=16)),
    (1024, dict(m=[4])),
    (16384, dict(m=[16, 4])),
    (256, dict(m=[4], max_levels=2)),
    (96, dict(m=[8])),
    (7, dict(m=[2])),
    (1, dict(m=[2])),
])
def test_hierarchy_matches_oracle(oracle, nt, kw):
    pr = W.Problem(1, 64, nt, 0.05, 3, 3, W.alpha_cfg12())
    sv = W.Solver(**kw)
    rc, h, _ = _create(pr, sv)
    assert rc == 0
    try:
        Ns, ms = _levels(h)
        oN, om = oracle.hierarchy(nt, sv)
        assert Ns == oN and ms == om
        nb = C.c_size_t()
        assert N.lib().slm_plan_workspace_size(h, C.byref(nb)) == 0
        assert nb.value >= 8 * nt * 64
    finally:
        N.lib().slm_plan_destroy(h)


@pytest.mark.parametrize("change,code", [
    (dict(dim=3), -2), (dict(nx=4), -2), (dict(nx=9000), -2), (dict(p=6), -2), (dict(r=0), -2),
    (dict(dt=0.0), -1), (dict(nt=0), -1), (dict(alpha=[]), -1),
    (dict(nt=65537), -2),                 # above the grid.y limit (SLM_MAX_NT)
    (dict(p=2), -2),                      # MGRIT needs odd p
])
def test_descriptor_validation(change, code):
    pr = W.Problem(1, 64, 64, 0.05, 3, 3, W.alpha_cfg12())
    sv = W.Solver(m=[4])
    for k, v in change.items():
        setattr(pr, k, v)
    rc, h, _ = _create(pr, sv)
    assert rc == code
    assert not h.value
    assert len(N.lib().slm_last_error(None)) > 0


@pytest.mark.parametrize("change", [dict(m=[1]), dict(gmres_kmax=11), dict(max_iter=0), dict(max_levels=0),
                                    dict(tol=-1.0)])
def test_solver_validation(change):
    pr = W.Problem(1, 64, 64, 0.05, 3, 3, W.alpha_cfg12())
    sv = W.Solver(m=[4])
    for k, v in change.items():
        setattr(sv, k, v)
    rc, h, _ = _create(pr, sv)
    assert rc == -1 and not h.value


def test_even_p_stepping_only_plan_is_valid():
    pr = W.Problem(1, 64, 64, 0.05, 2, 2, W.alpha_cfg12())
    rc, h, _ = _create(pr, W.Solver(m=[4], max_levels=1))
    assert rc == 0
    N.lib().slm_plan_destroy(h)


def test_calls_before_setup_fail_cleanly():
    pr = W.Problem(1, 64, 64, 0.05, 3, 3, W.alpha_cfg12())
    rc, h, _ = _create(pr, W.Solver(m=[4]))
    assert rc == 0
    try:
        st = N.Stats()
        assert N.lib().slm_solve(h, C.c_void_p(8), C.c_void_p(8), C.byref(st), None, 0, None) == -5
        assert N.lib().slm_step(h, C.c_void_p(8), C.c_void_p(8), 1, None) == -5
        assert N.lib().slm_plan_setup(h, None, 0, None) == -3
        assert N.lib().slm_plan_setup(h, C.c_void_p(1 << 20 | 8), 1 << 40, None) == -3   # misaligned
        assert b"aligned" in N.lib().slm_last_error(h)
    finally:
        N.lib().slm_plan_destroy(h)


def test_null_arguments():
    assert N.lib().slm_plan_create(None, None) == -1
    assert N.lib().slm_plan_workspace_size(None, None) == -1
    assert N.lib().slm_strerror(0) == b"ok"


def _bdesc(p=3, relax="FCF"):
    pr = W.Problem(1, 64, 32, 0.05, p, 3, W.alpha_cfg12())
    sv = W.Solver(m=[4], relax=relax)
    return N.make_desc(pr, sv, "fp64")


def test_batch_create_rejects_unsupported():
    """Batch descriptors are validated before any device call."""
    L = N.lib()
    h = C.c_void_p()
    assert L.slm_batch_create(None, 1, C.byref(h)) == -1
    d1, k1 = _bdesc()
    d2, k2 = _bdesc(p=2)
    arr = (N.Desc * 2)(d1, d2)
    assert L.slm_batch_create(arr, 2, C.byref(h)) == -2 and not h.value
    assert b"odd p" in L.slm_last_error(None)
    d3, k3 = _bdesc(relax="F")
    arr = (N.Desc * 2)(d1, d3)
    assert L.slm_batch_create(arr, 2, C.byref(h)) == -2
    arr = (N.Desc * 1)(d1)
    assert L.slm_batch_create(arr, 0, C.byref(h)) == -1
    assert L.slm_batch_setup(None, None, 0, None) == -1
    assert L.slm_batch_solve(None, None, None, None, None, 0, 0, None) == -1


def test_redisc_descriptor_validation():
    """The rediscretized coarse operator is FP64-only and has no adjoint;
    unknown coarse operators are rejected before any device call."""
    import dataclasses
    L = N.lib()
    pr = W.Problem(1, 64, 32, 0.05, 3, 3, W.alpha_cfg12())
    h = C.c_void_p()
    for sv, prec, adj, rc in [(W.Solver(m=[4], coarse_op="redisc"), "fp32", False, -2),
                              (W.Solver(m=[4], coarse_op="redisc"), "fp64", True, -2),
                              (W.Solver(m=[4], coarse_op="ideal"), "fp64", False, -2),
                              (W.Solver(m=[4], coarse_op="redisc"), "fp64", False, 0)]:
        d, k = N.make_desc(pr, sv, prec, adj)
        got = L.slm_plan_create(C.byref(d), C.byref(h))
        assert got == rc, (sv.coarse_op, prec, adj, got)
        if got == 0:
            L.slm_plan_destroy(h)
    # even p is allowed with the rediscretized operator (no D_{p+1} correction)
    d, k = N.make_desc(dataclasses.replace(pr, p=2), W.Solver(m=[4], coarse_op="redisc"), "fp64")
    assert L.slm_plan_create(C.byref(d), C.byref(h)) == 0
    L.slm_plan_destroy(h)


def test_fwd_euler_descriptor_validation():
    """The forward-Euler coarse operator (eq. Fp_def) is FP64-only, has no
    adjoint and, like the backward-Euler one, needs odd p."""
    import dataclasses
    L = N.lib()
    pr = W.Problem(1, 64, 32, 0.05, 3, 3, W.alpha_cfg12())
    h = C.c_void_p()
    sv = W.Solver(m=[4], coarse_op="fwd_euler")
    for prob, prec, adj, rc in [(pr, "fp32", False, -2), (pr, "fp64", True, -2),
                                (dataclasses.replace(pr, p=2), "fp64", False, -2), (pr, "fp64", False, 0)]:
        d, k = N.make_desc(prob, sv, prec, adj)
        got = L.slm_plan_create(C.byref(d), C.byref(h))
        assert got == rc, (prob.p, prec, adj, got)
        if got == 0:
            L.slm_plan_destroy(h)


@pytest.mark.parametrize("nx,nt,m", [(13, 24, [2, 3]), (20, 48, [4]), (64, 512, [8]), (100, 64, [4]),
                                     (512, 64, [8]), (1000, 16, [4]), (2048, 32, [8])])
def test_2d_per_block_slots_fit_the_workspace(nx, nt, m):
    """Sizing of the per-(interval, block) slot buffers of the 2D path, on
    the host: the batched kernels run ceil(S / 1024) workgroups per slice
    (at most 1024), and the workspace holds one residual partial per
    (interval, block) for the largest sweep and three GMRES partial sets of
    16 per (system, block) for the largest coarse sweep."""
    a, b = W.field_cfg3()
    pr = W.Problem(2, nx, nt, 2.0 * 2 / nx, 3, 3, a, b)
    rc, h, _ = _create(pr, W.Solver(m=m, coarsest_max_points=2))
    assert rc == 0
    try:
        S = nx * nx
        tiled, nb = C.c_int(), C.c_int()
        assert N.lib().slm_launch_info(h, 0, 1, C.byref(tiled), C.byref(nb)) == 0
        assert nb.value == min(1024, -(-S // 1024))
        Ns, ms = _levels(h)
        cap2 = max([Ns[l] // ms[l] for l in range(len(Ns)) if ms[l]] + [1])
        capg = max([Ns[l] // ms[l] for l in range(1, len(Ns)) if ms[l]] + [1])
        wsb = C.c_size_t()
        assert N.lib().slm_plan_workspace_size(h, C.byref(wsb)) == 0
        assert wsb.value >= 8 * nb.value * (cap2 + 3 * 16 * capg)
        # the level-0 step of a one-slice call over many tiles never exceeds them
        assert N.lib().slm_launch_info(h, len(Ns), 1, None, None) == -1
    finally:
        N.lib().slm_plan_destroy(h)


def test_autotune_needs_setup():
    pr = W.Problem(1, 64, 64, 0.05, 3, 3, W.alpha_cfg12())
    rc, h, _ = _create(pr, W.Solver(m=[4]))
    assert rc == 0
    try:
        assert N.lib().slm_autotune(h, None, 0, None, None) == -5
        assert N.lib().slm_autotune(None, None, 0, None, None) == -1
    finally:
        N.lib().slm_plan_destroy(h)
