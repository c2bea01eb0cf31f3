"""The paper's iteration counts (Tables 1-3) reproduced by the GPU solver on
every printed mesh, up to 2^12 x 2^14 in 1D and (2^9)^2 x 2^13 in 2D, in
FP64.  The initial iterate is random (its distribution is not given in the
paper; here U[0, 1) at the C-points) and so are the ERK tableaux for r = 3, 5,
so a count may differ from the printed one by one cycle; the rediscretised
counts, where the solver is close to stagnation, by 5% (at least 2)."""
import time

import pytest

import paper_tables as PT

pytestmark = pytest.mark.gpu

_ROWS = PT.rows()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _iterations(torch, row, coarse_op="modified"):
    from paper_2203_13382_amd import Plan
    pr, u0 = PT.problem(row)
    plan = Plan(pr, PT.solver(row, coarse_op), "fp64").setup()
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    c = torch.rand((plan.n_cpoints, pr.S), generator=g, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    st, hist = plan.solve_cpoints(torch.from_numpy(u0), c)
    print(f"{PT.row_id(row)} {coarse_op}: {st['iterations']} cycles ({st['status']}), "
          f"printed {row['redisc'] if coarse_op == 'redisc' else row['iters']}, "
          f"{time.perf_counter() - t0:.2f} s", flush=True)
    assert st["status"] == "converged", st
    return st["iterations"]


@pytest.mark.parametrize("row", _ROWS, ids=PT.row_id)
def test_paper_iteration_counts(torch, row):
    it = _iterations(torch, row)
    assert abs(it - row["iters"]) <= 1, (row, it)


@pytest.mark.parametrize("row", [r for r in _ROWS if r["redisc"] is not None],
                         ids=lambda r: PT.row_id(r, "T3redisc"))
def test_paper_rediscretised_counts(torch, row):
    it = _iterations(torch, row, "redisc")
    assert abs(it - row["redisc"]) <= max(2, 0.05 * row["redisc"]), (row, it)
