"""GPU parity of the 2D path (tensor-product SL step, bilinear backtracking,
eq. BEOper_2D with batched GMRES) against the FP64 oracle, through the C ABI.
"""
import numpy as np
import pytest

from paper_2203_13382_amd import inputs as I
from paper_2203_13382_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cfg3_field_p5":
        a, b = W.field_cfg3()
        pr = W.Problem(2, 16, 32, 2.0 * 2 / 16, 5, 5, a, b)
        sv = W.Solver(m=[4], coarsest_max_points=2, gmres_rtol=1e-2)
    elif name == "cfg5_field_p3":
        a, b = W.field_cfg5((1.0, 0.3, 1.0, 0.2))
        pr = W.Problem(2, 24, 48, 2.0 * 2 / 24, 3, 3, a, b)
        sv = W.Solver(m=[4], coarsest_max_points=2, gmres_rtol=1e-2)
    elif name == "ragged_p1_f":
        a, b = W.field_cfg3()
        pr = W.Problem(2, 20, 24, 1.7 * 2 / 20, 1, 1, a, b)
        sv = W.Solver(m=[2, 3], coarsest_max_points=2, relax="F", gmres_rtol=0.0)
    elif name == "two_level_p3":
        kt = 2.0 / 3.4
        a = [W.term(0.5, kt=kt), W.term(-0.5, ky=2.0, kt=kt)]
        b = [W.term(-0.5, kt=kt), W.term(-0.5, kx=2.0, kt=kt)]
        pr = W.Problem(2, 32, 32, 0.85 * 2 / 32, 3, 3, a, b)
        sv = W.Solver(m=[4], max_levels=2, gmres_rtol=0.0)
    else:
        raise KeyError(name)
    return pr, sv


CASES = ["cfg3_field_p5", "cfg5_field_p3", "ragged_p1_f", "two_level_p3"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


_cache = {}


def _setup(name, oracle, precision="fp64"):
    key = (name, precision)
    if key not in _cache:
        from paper_2203_13382_amd import Plan
        pr, sv = _case(name)
        plan = Plan(pr, sv, precision).setup()
        ctx = oracle.Context(pr, sv)
        _cache[key] = (pr, sv, plan, ctx)
    return _cache[key]


def _rel(a, b):
    return np.abs(a - b).max() / max(1e-300, np.abs(b).max())


@pytest.mark.parametrize("name", CASES)
def test_setup_arrays(name, oracle, torch):
    pr, sv, plan, ctx = _setup(name, oracle)
    assert plan.N == ctx.N
    h = pr.h
    idx = np.arange(pr.S)
    X = -1 + (idx % pr.nx) * h
    Y = -1 + (idx // pr.nx) * h
    for l in range(plan.L):
        disp, sig = plan.level_arrays(l)
        dx, dy = disp[0].cpu().numpy(), disp[1].cpu().numpy()
        rx = (X[None, :] - ctx.dep(l, 0)) / h
        ry = (Y[None, :] - ctx.dep(l, 1)) / h
        scale = max(1.0, np.abs(rx).max(), np.abs(ry).max())
        assert np.abs(dx - rx).max() < 1e-9 * scale and np.abs(dy - ry).max() < 1e-9 * scale, l
        if l > 0:
            for comp in (0, 1):
                s_g = sig[comp].cpu().numpy()
                s_o = ctx.sigma(l, comp)
                assert np.abs(s_g - s_o).max() < 1e-9 * max(1.0, np.abs(s_o).max()), (l, comp)


@pytest.mark.parametrize("name", CASES)
def test_apply_phi_every_level(name, oracle, torch):
    pr, sv, plan, ctx = _setup(name, oracle)
    rng = np.random.default_rng(7)
    for l in range(plan.L):
        cnt = min(plan.N[l], 5)
        n0 = plan.N[l] - cnt
        xin = rng.standard_normal((cnt, pr.S))
        out = plan.apply_phi(l, n0, torch.from_numpy(xin)).cpu().numpy()
        ref = np.stack([ctx.apply_phi(l, n0 + k, xin[k]) for k in range(cnt)])
        # rtol = 0: GMRES past convergence, see test_gpu_1d._phi_tol
        tol = 1e-7 if l > 0 and sv.gmres_rtol == 0.0 else 1e-11
        assert _rel(out, ref) < tol, (l, _rel(out, ref))


@pytest.mark.parametrize("name", CASES)
def test_sequential_stepping(name, oracle, torch):
    pr, sv, plan, ctx = _setup(name, oracle)
    u0 = I.initial_condition(pr, 0)
    u = plan.step(torch.from_numpy(u0)).cpu().numpy()
    ref = oracle.seq_fine(pr, u0)
    assert _rel(u, ref) < 1e-11
    last = plan.step(torch.from_numpy(u0), store_all=False).cpu().numpy()
    assert np.array_equal(last, u[-1])


def _ora_chain(ctx, l, start, n_first, nsteps, g):
    v = start.copy()
    out = []
    for k in range(nsteps):
        v = ctx.apply_phi(l, n_first + k, v)
        if g is not None:
            v = v + g[n_first + k + 1]
        out.append(v)
    return out


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("level", [0, 1])
def test_relaxation_sweeps(name, level, oracle, torch):
    pr, sv, plan, ctx = _setup(name, oracle)
    if level >= plan.L - 1:
        pytest.skip("no coarser level below")
    Nl, m = plan.N[level], plan.m[level]
    nc = Nl // m
    rng = np.random.default_rng(11 + level)
    cin = rng.standard_normal((nc + 1, pr.S))
    g = rng.standard_normal((Nl + 1, pr.S)) if level > 0 else None
    tg = None if g is None else torch.from_numpy(g)
    cout = plan.relax(level, "FC", torch.from_numpy(cin), tg).cpu().numpy()
    ref = np.zeros_like(cin)
    ref[0] = cin[0]
    for j in range(nc):
        ref[j + 1] = _ora_chain(ctx, level, cin[j], j * m, m, g)[-1]
    assert _rel(cout, ref) < 1e-11
    res, nrm = plan.relax(level, "RES", torch.from_numpy(cin), tg)
    res = res.cpu().numpy()
    rref = np.stack([_ora_chain(ctx, level, cin[j], j * m, m, g)[-1] - cin[j + 1] for j in range(nc)])
    assert _rel(res[1:], rref) < 1e-11
    assert abs(nrm - np.linalg.norm(rref)) < 1e-11 * np.linalg.norm(rref)
    v = plan.relax(level, "F", torch.from_numpy(cin), tg).cpu().numpy()
    vref = np.zeros((Nl + 1, pr.S))
    for j in range(nc):
        vref[j * m] = cin[j]
        for k, s in enumerate(_ora_chain(ctx, level, cin[j], j * m, m - 1, g)):
            vref[j * m + k + 1] = s
    vref[Nl] = cin[nc]
    assert _rel(v, vref) < 1e-11


@pytest.mark.parametrize("name", CASES)
def test_mgrit_solve(name, oracle, torch):
    pr, sv, plan, ctx = _setup(name, oracle)
    u0 = I.initial_condition(pr, 0)
    ui = I.initial_iterate(pr.nt, pr.S, plan.m[0], 1)
    u_ref, st_ref, h_ref = ctx.mgrit(u0, ui)
    u = torch.from_numpy(ui).cuda()
    st, hist = plan.solve(torch.from_numpy(u0), u)
    assert st["status"] == st_ref["status"]
    assert st["iterations"] == st_ref["iterations"]
    assert np.abs(hist - h_ref).max() <= 1e-8 * h_ref[0]
    big = h_ref > 1e-7 * h_ref[0]
    assert np.abs(hist[big] / h_ref[big] - 1).max() < 1e-6
    assert st["gmres_solves"] == st_ref["gmres_solves"]
    assert abs(st["gmres_iters"] - st_ref["gmres_iters"]) <= 3 * sv.gmres_kmax
    assert _rel(u.cpu().numpy(), u_ref) < 1e-9
    u2 = torch.from_numpy(ui).cuda()
    st2, hist2 = plan.solve(torch.from_numpy(u0), u2)
    assert torch.equal(u, u2) and np.array_equal(hist, hist2)


# FP32-bulk error bounds against the FP64 oracle (stepping, MGRIT to a
# relative 1e-6): about three times the errors measured on MI355X.
# Measured: cfg3_field_p5 7.6e-7 / 7.6e-7, cfg5_field_p3 2.7e-7 / 2.7e-7.
FP32_BOUND = {"cfg3_field_p5": (2.5e-6, 2.5e-6), "cfg5_field_p3": (1e-6, 1e-6)}


@pytest.mark.parametrize("name", ["cfg3_field_p5", "cfg5_field_p3"])
def test_fp32_bulk(name, oracle, torch):
    pr, sv, plan, ctx = _setup(name, oracle, "fp32")
    u0 = I.initial_condition(pr, 0)
    useq = oracle.seq_fine(pr, u0)
    u = plan.step(torch.from_numpy(u0)).cpu().numpy()
    e_step = _rel(u, useq)
    print(f"{name} fp32 stepping: rel. error {e_step:.2e}")
    assert e_step < FP32_BOUND[name][0]
    import dataclasses
    from paper_2203_13382_amd import Plan
    p32 = Plan(pr, dataclasses.replace(sv, tol=1e-6), "fp32").setup()
    ui = I.initial_iterate(pr.nt, pr.S, plan.m[0], 1).astype(np.float32)
    uu = torch.from_numpy(ui).cuda()
    st, hist = p32.solve(torch.from_numpy(u0.astype(np.float32)), uu)
    assert st["status"] in ("converged", "stagnated")
    e_mg = _rel(uu.cpu().numpy(), useq)
    print(f"{name} fp32 MGRIT to rel. 1e-6: rel. error {e_mg:.2e}")
    assert e_mg < FP32_BOUND[name][1]
