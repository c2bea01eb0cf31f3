"""slm_relax_noalloc (the relaxation sweep for callers that cannot allocate)
against slm_relax through the C ABI: identical outputs, bit for bit (same
kernels and summation order), on consecutive calls whose second input is
smaller, and its size limit reported as an error without a launch."""
import ctypes as C

import numpy as np
import pytest

from paper_2203_13382_amd import _native as N
from paper_2203_13382_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _sweeps(torch, plan, level, fn, seed):
    """Run the three sweep kinds of level ``level`` through ``fn`` (the C
    entry point) on seeded inputs; returns their outputs and the norm."""
    S, Nl, m = plan.S, plan.N[level], plan.m[level]
    nc = Nl // m
    rng = np.random.default_rng(seed)
    cin = torch.from_numpy(rng.standard_normal((nc + 1, S))).to("cuda", plan.dtype)
    g = None if level == 0 else torch.from_numpy(rng.standard_normal((Nl + 1, S))).to("cuda", plan.dtype)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    cout = torch.zeros(nc + 1, S, dtype=plan.dtype, device="cuda")
    res = torch.zeros(nc + 1, S, dtype=plan.dtype, device="cuda")
    v = torch.zeros(Nl + 1, S, dtype=plan.dtype, device="cuda")
    norm = C.c_double(0.0)
    N.check(fn(plan.h, level, N.SWEEP["FC"], _ptr(g), _ptr(cin), _ptr(cout), None, None, None, st), plan.h)
    N.check(fn(plan.h, level, N.SWEEP["RES"], _ptr(g), _ptr(cin), None, _ptr(res), None, C.byref(norm), st), plan.h)
    N.check(fn(plan.h, level, N.SWEEP["F"], _ptr(g), _ptr(cin), None, None, _ptr(v), None, st), plan.h)
    torch.cuda.synchronize()
    return cout.cpu().numpy(), res.cpu().numpy(), v.cpu().numpy(), norm.value


def _plan(pr, sv, prec="fp64"):
    from paper_2203_13382_amd import Plan
    return Plan(pr, sv, prec).setup()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_relax_on_two_calls(torch, prec):
    lib = N.lib()
    big = _plan(W.Problem(1, 1024, 2048, 4 * 2 / 1024, 3, 3, W.alpha_cfg12()),
                W.Solver(m=[8], coarsest_max_points=16, gmres_rtol=1e-2), prec)
    small = _plan(W.Problem(1, 200, 96, 0.85 * 2 / 200, 5, 5, W.alpha_cfg12(0.3)),
                  W.Solver(m=[4], coarsest_max_points=2, gmres_rtol=1e-2), prec)
    # first call: the larger input (256 intervals on level 0), then a smaller one
    for plan, level, seed in [(big, 0, 1), (big, 1, 2), (small, 0, 3), (small, 1, 4)]:
        ref = _sweeps(torch, plan, level, lib.slm_relax, seed)
        got = _sweeps(torch, plan, level, lib.slm_relax_noalloc, seed)
        for a, b in zip(ref[:3], got[:3]):
            assert np.array_equal(a, b)
        assert ref[3] == got[3] and ref[3] > 0.0


def test_noalloc_limits(torch):
    lib = N.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # more intervals than the static scratch holds: an error, nothing launched
    pr = W.Problem(1, 8, 2 * 16385, 0.01, 1, 1, [W.term(1.0)])
    plan = _plan(pr, W.Solver(m=[2], max_levels=2))
    assert plan.N[0] // plan.m[0] == 16385
    res = torch.zeros(16386, 8, dtype=torch.float64, device="cuda")
    cin = torch.zeros(16386, 8, dtype=torch.float64, device="cuda")
    rc = lib.slm_relax_noalloc(plan.h, 0, N.SWEEP["RES"], None, _ptr(cin), None, _ptr(res), None, None, st)
    assert rc == -1 and b"16384" in lib.slm_last_error(plan.h)
    # 2D plans are not supported by the allocation-free variant
    a, b = W.field_cfg3()
    p2 = _plan(W.Problem(2, 16, 16, 0.1, 1, 1, a, b), W.Solver(m=[4], max_levels=2))
    rc = lib.slm_relax_noalloc(p2.h, 0, N.SWEEP["FC"], None, None, _ptr(cin), None, None, None, st)
    assert rc == -2
