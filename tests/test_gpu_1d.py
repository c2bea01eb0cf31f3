"""GPU parity of the 1D path against the FP64 oracle, element by element,
through the C ABI.

Cases span several workgroup tiles, ragged spatial sizes (nx not a multiple
of 64), every interpolation order used by MGRIT, two-level and multilevel
hierarchies, F and FCF relaxation, and FP32 bulk.
"""
import numpy as np
import pytest

from paper_2203_13382_amd import inputs as I
from paper_2203_13382_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cfg1":
        pr, sv, _ = W.config(1)
    elif name == "cfg2_small":
        pr, sv, _ = W.config(2)
        pr = W.scaled(pr, 512, 2048, 4.0)
    elif name == "ragged_p5":
        pr = W.Problem(1, 200, 96, 2.3 * 2 / 200, 5, 5, W.alpha_cfg12(0.3))
        sv = W.Solver(m=[4], coarsest_max_points=2, gmres_rtol=1e-2)
    elif name == "ept2_mixed_m":
        pr = W.Problem(1, 1500, 64, 3.1 * 2 / 1500, 3, 3, W.alpha_cfg12())
        sv = W.Solver(m=[4, 2], coarsest_max_points=2, gmres_rtol=1e-2)
    elif name == "ept4_f_relax":
        pr = W.Problem(1, 4096, 48, 4.0 * 2 / 4096, 3, 3, W.alpha_cfg12())
        sv = W.Solver(m=[4], coarsest_max_points=2, relax="F", gmres_rtol=0.0)
    elif name == "ept8_p1":
        pr = W.Problem(1, 8192, 16, 0.85 * 2 / 8192, 1, 1, [W.term(1.0), W.term(0.4, kx=2.0, kt=1.0)])
        sv = W.Solver(m=[4], max_levels=2, gmres_rtol=1e-2)
    else:
        raise KeyError(name)
    return pr, sv


CASES = ["cfg1", "cfg2_small", "ragged_p5", "ept2_mixed_m", "ept4_f_relax", "ept8_p1"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def built():
    from paper_2203_13382_amd import _native
    _native.lib()
    return True


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
def test_setup_arrays(name, oracle, torch, built):
    pr, sv, plan, ctx = _setup(name, oracle)
    assert plan.N == ctx.N and plan.m == ctx.m[:len(plan.m)]
    x = I.mesh(pr.nx)
    for l in range(plan.L):
        disp, sig = plan.level_arrays(l)
        d_gpu = disp[0].cpu().numpy()
        d_ora = (x[None, :] - ctx.dep(l)) / pr.h
        assert np.abs(d_gpu - d_ora).max() < 1e-9 * max(1.0, np.abs(d_ora).max()), l
        if l > 0:
            s_gpu = sig[0].cpu().numpy()
            s_ora = ctx.sigma(l)
            assert np.abs(s_gpu - s_ora).max() < 1e-9 * max(1.0, np.abs(s_ora).max()), l


def _phi_tol(sv, level):
    """Agreement of one level step with the oracle's.  With rtol = 0 GMRES
    keeps iterating after it has converged; the Krylov basis of one-pass
    Gram-Schmidt then loses orthogonality, and the Pythagorean norm amplifies
    that loss by ||w||^2 / hn^2 (at most 1e3 before the explicit norm takes
    over), so the two sides' roundings of it part at about 1e-8."""
    return 1e-7 if level > 0 and sv.gmres_rtol == 0.0 else 1e-11


@pytest.mark.parametrize("name", CASES)
def test_apply_phi_every_level(name, oracle, torch, built):
    pr, sv, plan, ctx = _setup(name, oracle)
    rng = np.random.default_rng(7)
    for l in range(plan.L):
        cnt = min(plan.N[l], 6)
        n0 = plan.N[l] - cnt
        xin = rng.standard_normal((cnt, pr.S))
        out = plan.apply_phi(l, n0, torch.from_numpy(xin)).cpu().numpy()
        ref = np.stack([ctx.apply_phi(l, n0 + k, xin[k]) for k in range(cnt)])
        assert _rel(out, ref) < _phi_tol(sv, l), (l, _rel(out, ref))


@pytest.mark.parametrize("name", CASES)
def test_sequential_stepping(name, oracle, torch, built):
    pr, sv, plan, ctx = _setup(name, oracle)
    u0 = I.initial_condition(pr, 0)
    u = plan.step(torch.from_numpy(u0)).cpu().numpy()
    ref = oracle.seq_fine(pr, u0)
    assert _rel(u, ref) < 1e-11
    last = plan.step(torch.from_numpy(u0), store_all=False).cpu().numpy()
    assert np.array_equal(last, u[-1])


def _ora_chain(ctx, l, start, n_first, nsteps, g):
    v = start.copy()
    states = []
    for k in range(nsteps):
        v = ctx.apply_phi(l, n_first + k, v)
        if g is not None:
            v = v + g[n_first + k + 1]
        states.append(v)
    return states


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("level", [0, 1])
def test_relaxation_sweeps(name, level, oracle, torch, built):
    pr, sv, plan, ctx = _setup(name, oracle)
    if level >= plan.L - 1:
        pytest.skip("no coarser level below")
    Nl, m = plan.N[level], plan.m[level]
    nc = Nl // m
    rng = np.random.default_rng(11 + level)
    cin = rng.standard_normal((nc + 1, pr.S))
    g = rng.standard_normal((Nl + 1, pr.S)) if level > 0 else None
    tg = None if g is None else torch.from_numpy(g)
    # F then C relaxation
    cout = plan.relax(level, "FC", torch.from_numpy(cin), tg).cpu().numpy()
    ref = np.zeros_like(cin)
    ref[0] = cin[0]
    for j in range(nc):
        ref[j + 1] = _ora_chain(ctx, level, cin[j], j * m, m, g)[-1]
    assert _rel(cout, ref) < 1e-11
    # F-relaxation + C-point residual and its norm
    res, nrm = plan.relax(level, "RES", torch.from_numpy(cin), tg)
    res = res.cpu().numpy()
    rref = np.zeros_like(cin)
    for j in range(nc):
        rref[j + 1] = _ora_chain(ctx, level, cin[j], j * m, m, g)[-1] - cin[j + 1]
    assert _rel(res[1:], rref[1:]) < 1e-11
    assert abs(nrm - np.linalg.norm(rref[1:])) < 1e-11 * np.linalg.norm(rref[1:])
    # F-relaxation writing every point
    v = plan.relax(level, "F", torch.from_numpy(cin), tg).cpu().numpy()
    vref = np.zeros((Nl + 1, pr.S))
    for j in range(nc):
        vref[j * m] = cin[j]
        st = _ora_chain(ctx, level, cin[j], j * m, m - 1, g)
        for k, s in enumerate(st):
            vref[j * m + k + 1] = s
    vref[Nl] = cin[nc]
    assert _rel(v, vref) < 1e-11


@pytest.mark.parametrize("name", CASES)
def test_mgrit_solve(name, oracle, torch, built):
    """Same iteration count and residual history as the oracle; the result
    agrees with the oracle's MGRIT result and with sequential stepping."""
    pr, sv, plan, ctx = _setup(name, oracle)
    u0 = I.initial_condition(pr, 0)
    ui = I.initial_iterate(pr.nt, pr.S, plan.m[0] if plan.L > 1 else 1, 1)
    u_ref, st_ref, h_ref = ctx.mgrit(u0, ui)
    u = torch.from_numpy(ui).cuda()
    st, hist = plan.solve(torch.from_numpy(u0), u)
    assert st["status"] == st_ref["status"]
    assert st["iterations"] == st_ref["iterations"]
    assert st["n_levels"] == st_ref["n_levels"]
    if plan.L > 1:
        assert np.abs(hist - h_ref).max() <= 1e-8 * h_ref[0] + 1e-12 * np.abs(h_ref).max()
        # relative agreement where rho_k is far above its rounding floor
        # (~1e-16 * ||u|| * sqrt(#entries)); deeper entries are covered by
        # the absolute bound above
        big = h_ref > 1e-7 * h_ref[0]
        assert np.abs(hist[big] / h_ref[big] - 1).max() < 1e-6
        assert st["gmres_solves"] == st_ref["gmres_solves"]
        # C-points that are already exact leave residuals of pure rounding
        # noise (|b| ~ 1e-17); one side may get exactly zero there and skip
        # that B-solve's iterations, so allow a few solves' worth of difference.
        assert abs(st["gmres_iters"] - st_ref["gmres_iters"]) <= 3 * sv.gmres_kmax
    uc = u.cpu().numpy()
    assert _rel(uc, u_ref) < 1e-9
    # determinism: a second solve from the same input is bitwise identical
    u2 = torch.from_numpy(ui).cuda()
    st2, hist2 = plan.solve(torch.from_numpy(u0), u2)
    assert torch.equal(u, u2) and np.array_equal(hist, hist2)


# FP32-bulk error bounds against the FP64 oracle (stepping, MGRIT to a
# relative 1e-6): about three times the errors measured on MI355X.
# Measured: cfg1 3.7e-7 / 4.8e-6, cfg2_small 5.8e-6 / 1.3e-5, ragged_p5
# 2.8e-6 / 5.0e-6.
FP32_BOUND = {"cfg1": (1.2e-6, 1.5e-5), "cfg2_small": (1.8e-5, 4e-5), "ragged_p5": (9e-6, 1.5e-5)}


@pytest.mark.parametrize("name", ["cfg1", "cfg2_small", "ragged_p5"])
def test_fp32_bulk(name, oracle, torch, built):
    """FP32 bulk (FP64 tracing, sigma, inner products and norms): stepping
    and MGRIT agree with the FP64 oracle to FP32 accuracy."""
    pr, sv, plan, ctx = _setup(name, oracle, "fp32")
    _, _, plan64, _ = _setup(name, oracle, "fp64")
    d32 = plan.level_arrays(0)[0].cpu().numpy()
    d64 = plan64.level_arrays(0)[0].cpu().numpy()
    assert np.abs(d32 - d64).max() <= 1e-6 * max(1.0, np.abs(d64).max())
    for l in range(1, plan.L):
        assert torch.equal(plan.level_arrays(l)[1], plan64.level_arrays(l)[1])
    u0 = I.initial_condition(pr, 0)
    useq = oracle.seq_fine(pr, u0)
    u = plan.step(torch.from_numpy(u0)).cpu().numpy()
    e_step = _rel(u, useq)
    print(f"{name} fp32 stepping: rel. error {e_step:.2e}")
    assert e_step < FP32_BOUND[name][0]
    if plan.L > 1:
        ui = I.initial_iterate(pr.nt, pr.S, plan.m[0], 1).astype(np.float32)
        uu = torch.from_numpy(ui).cuda()
        import dataclasses
        sv32 = dataclasses.replace(sv, tol=1e-6, tol_mode="rel")
        from paper_2203_13382_amd import Plan
        p32 = Plan(pr, sv32, "fp32").setup()
        st, hist = p32.solve(torch.from_numpy(u0.astype(np.float32)), uu)
        assert st["status"] in ("converged", "stagnated")
        e_mg = _rel(uu.cpu().numpy(), useq)
        print(f"{name} fp32 MGRIT to rel. 1e-6: rel. error {e_mg:.2e}")
        assert e_mg < FP32_BOUND[name][1]


def test_setup_refuses_nt_above_grid_y(torch, built):
    # launches put time steps on grid.y: setup refuses more steps than the
    # device reports for it (65536 on MI355X), before launching anything
    from paper_2203_13382_amd import Plan
    from paper_2203_13382_amd._native import NativeError
    pr = W.Problem(1, 8, 65537, 0.01, 1, 1, [W.term(1.0)])
    with pytest.raises(NativeError, match="grid.y"):
        Plan(pr, W.Solver(m=[2], max_levels=2)).setup()
    pr = W.Problem(1, 8, 65536, 0.01, 1, 1, [W.term(1.0)])
    plan = Plan(pr, W.Solver(m=[2], max_levels=2)).setup()
    assert plan.N[0] == 65536
