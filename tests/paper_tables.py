"""The paper's iteration-count experiments (Tables 1-3): the printed counts
from tests/golden/paper_iterations.txt and the problem and solver each cell
describes.  Used by the oracle's pins and by the GPU reproduction."""
import os

from paper_2203_13382_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_iterations.txt")


def rows():
    out = []
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        m = [int(x) for x in f[5].split(",")] if "," in f[5] else int(f[5])
        out.append(dict(table=f[0], field=f[1], p=int(f[2]), nx=int(f[3]), nt=int(f[4]), m=m,
                        iters=int(f[6]), redisc=int(f[7]) if len(f) > 7 else None))
    return out


def row_id(r, prefix=""):
    m = "-".join(str(x) for x in r["m"]) if isinstance(r["m"], list) else r["m"]
    return f"{prefix or r['table']}-{r['field']}-p{r['p']}-nx{r['nx']}-m{m}"


def problem(row):
    """The cell's problem and initial condition (workloads.paper_problem)."""
    dim = 2 if row["table"] == "T3" else 1
    pr = W.paper_problem(dim, row["field"], row["p"], row["nx"], row["nt"])
    return pr, W.paper_initial_condition(dim, row["nx"])


def solver(row, coarse_op="modified"):
    """Table 1: two levels, coarse operator of eq. (Psi_Bp_def2) with exactly
    10 GMRES iterations; Tables 2 and 3 and the Sec. 5 runs: V-cycles down to
    2 points, GMRES to relative residual 1e-2 or 10 iterations; m on every
    level (Sec. 5: 16 on the first, 4 below); stop at a relative residual of
    1e-10."""
    if row["table"] == "T1":
        return W.Solver(m=[row["m"]], max_levels=2, gmres_kmax=10, gmres_rtol=0.0, max_iter=300)
    m = row["m"] if isinstance(row["m"], list) else [row["m"]]
    return W.Solver(m=m, coarsest_max_points=2, gmres_kmax=10, gmres_rtol=1e-2,
                    max_iter=300, coarse_op=coarse_op)
