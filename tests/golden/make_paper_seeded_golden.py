"""Write tests/golden/paper_seeded_oracle.txt: the oracle's MGRIT runs of the
paper's iteration-count experiments, started from the seeded initial iterate
(slmo_seeded_iterate, seed 5), so that the GPU can be compared with them
cycle by cycle on identical inputs.

Cells: Tables 1 and 2 on the 2^8 x 2^10 mesh (every alpha, p and m), and
Table 3 on the (2^6)^2 x 2^10 mesh with the modified coarse operator and
with the rediscretized one (the counts in parentheses).  Each line holds the
cell, the iteration count, the status, the number of coarse solves and of
GMRES iterations, and the residual history rho_k.

Only the oracle is called.  Run from the repository root:
    python tests/golden/make_paper_seeded_golden.py [workers]
"""
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

SEED = 5
OUT = os.path.join(HERE, "paper_seeded_oracle.txt")


def cells():
    import paper_tables as PT
    out = []
    for r in PT.rows():
        if r["table"] in ("T1", "T2") and r["nx"] == 256:
            out.append((r, "modified"))
        if r["table"] == "T3" and r["nx"] == 64:
            out.append((r, "modified"))
            if r["redisc"] is not None:
                out.append((r, "redisc"))
    return out


def run(cell):
    import paper_tables as PT
    from oracle import oracle as O
    r, op = cell
    pr, u0 = PT.problem(r)
    ctx = O.Context(pr, PT.solver(r, op))
    m0 = r["m"] if isinstance(r["m"], int) else r["m"][0]
    ui = O.seeded_iterate(SEED, pr.nt, pr.S, m0)
    _, st, hist = ctx.mgrit(u0, ui)
    m = "-".join(str(x) for x in r["m"]) if isinstance(r["m"], list) else str(r["m"])
    head = (f"{r['table']} {r['field']} {r['p']} {r['nx']} {r['nt']} {m} {op} {SEED} {st['iterations']} "
            f"{st['status']} {st['gmres_solves']} {st['gmres_iters']}")
    line = head + " " + " ".join(f"{h:.17g}" for h in hist)
    print(head, flush=True)
    return line


def main():
    from oracle import oracle as O
    O.build(force=False)
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    cs = cells()
    # the slow 2D cells first, so that the pool stays busy to the end
    order = sorted(range(len(cs)), key=lambda i: (cs[i][0]["table"] != "T3", -cs[i][0]["p"]))
    with mp.Pool(workers) as pool:
        lines = pool.map(run, [cs[i] for i in order], chunksize=1)
    res = [None] * len(cs)
    for k, i in enumerate(order):
        res[i] = lines[k]
    with open(OUT, "w") as f:
        f.write("# Oracle MGRIT runs of the paper's iteration-count cells from the seeded\n"
                "# initial iterate (seed 5); written by make_paper_seeded_golden.py.\n"
                "#   table field p nx nt m coarse_op seed iterations status gmres_solves gmres_iters\n"
                "#   rho_0 rho_1 ...\n")
        for line in res:
            f.write(line + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
