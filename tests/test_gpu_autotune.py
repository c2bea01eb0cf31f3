"""slm_autotune: every launch shape it may choose gives bitwise the same
results (2D level-0 tile shapes of the LDS-staged SL step, 1D elements per
thread and slice double-buffering of the level-0 sweeps without a
residual), and the choice is read from / appended to the cache file."""
import numpy as np
import pytest

from paper_2203_13382_amd import inputs as I
from paper_2203_13382_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _key(plan, pr):
    return (f"plan dim={pr.dim} nx={pr.nx} nt={pr.nt} p={pr.p} r={pr.r} prec={0 if plan.precision == 'fp64' else 1} "
            f"m0={plan.m[0]} levels={plan.L}")


def _run(torch, plan, pr, seed=3):
    nc = plan.N[0] // plan.m[0]
    rng = np.random.default_rng(seed)
    cin = torch.from_numpy(rng.standard_normal((nc + 1, pr.S))).to("cuda", plan.dtype)
    cout = plan.relax(0, "FC", cin).cpu().numpy()
    res, nrm = plan.relax(0, "RES", cin)
    v = plan.relax(0, "F", cin).cpu().numpy()
    u = torch.zeros((pr.nt + 1, pr.S), dtype=plan.dtype, device="cuda")
    plan.seed_iterate(u, 7)
    st, hist = plan.solve(torch.from_numpy(I.initial_condition(pr, 0)), u)
    return cout, res.cpu().numpy(), nrm, v, u.cpu().numpy(), hist, st["iterations"]


def _same(a, b):
    for x, y in zip(a, b):
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y)
        else:
            assert x == y


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_2d_tile_shapes_are_bitwise_equal(torch, tmp_path, prec):
    from paper_2203_13382_amd import Plan
    a, b = W.field_cfg3()
    pr = W.Problem(2, 256, 128, 2.0 * 2 / 256, 5, 5, a, b)
    sv = W.Solver(m=[4], coarsest_max_points=16, gmres_rtol=1e-2, tol=1e-10 if prec == "fp64" else 1e-6)
    plan = Plan(pr, sv, prec).setup()
    ref = None
    for tile in range(4):
        cache = tmp_path / f"tile{tile}.txt"
        cache.write_text(f"{_key(plan, pr)} | tile={tile} ept=0 dbuf=-1\n")
        plan.autotune(cache)
        # the shape is used when its window fits (FP64 128x32 exceeds 48 KB of LDS)
        assert plan.launch_info(0, plan.N[0] // plan.m[0])[0] in (1 + tile, 0)
        out = _run(torch, plan, pr)
        if ref is None:
            ref = out
        else:
            _same(out, ref)


def test_1d_level0_shapes_are_bitwise_equal(torch, tmp_path):
    from paper_2203_13382_amd import Plan
    pr = W.Problem(1, 4096, 2048, 4 * 2 / 4096, 3, 3, W.alpha_cfg12())
    sv = W.Solver(m=[8], coarsest_max_points=16, gmres_rtol=1e-2, tol=1e-10)
    plan = Plan(pr, sv, "fp64").setup()
    ref = None
    for ept, dbuf in [(0, -1), (4, 0), (4, 1), (8, 0), (8, 1)]:
        cache = tmp_path / f"e{ept}d{dbuf}.txt"
        cache.write_text(f"{_key(plan, pr)} | tile=0 ept={ept} dbuf={dbuf}\n")
        plan.autotune(cache)
        out = _run(torch, plan, pr)
        if ref is None:
            ref = out
        else:
            _same(out, ref)


def test_autotune_measures_then_reads_the_cache(torch, tmp_path):
    from paper_2203_13382_amd import Plan
    pr = W.Problem(1, 2048, 1024, 4 * 2 / 2048, 3, 3, W.alpha_cfg12())
    plan = Plan(pr, W.Solver(m=[8], coarsest_max_points=16, gmres_rtol=1e-2), "fp64").setup()
    cache = tmp_path / "tune.txt"
    plan.autotune(cache)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith(_key(plan, pr) + " |")
    plan.autotune(cache)                      # read back, nothing appended
    assert cache.read_text().splitlines() == lines
    plan.autotune()                           # no cache: measure only
