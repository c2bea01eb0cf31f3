"""Writes tests/golden/adjoint_oracle.txt: the FP64 oracle's loss and
gradient for the 2D adjoint workload at full size (workloads.adjoint_config:
256^2, nt = 2048, dt = 2h, p = r = 3, field_cfg5(theta); u_obs from
sequential stepping at theta_true; u0 = seeded Fourier IC, seed 0):
L = 1/2 ||u_nt - u_obs||^2, dL/dtheta (4 coefficients) and 256 sampled
entries of dL/du0, by sequential stepping, the sequential adjoint sweep and
the coefficient gradient of oracle/.  Calls only oracle/ and the seeded
input generators.

    python tests/golden/make_adjoint_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2203_13382_amd import inputs as I  # noqa: E402
from paper_2203_13382_amd import workloads as W  # noqa: E402


def with_theta(pr, th):
    import dataclasses
    na = len(pr.alpha)
    al = [(float(th[k]),) + tuple(t[1:]) for k, t in enumerate(pr.alpha)]
    be = [(float(th[na + k]),) + tuple(t[1:]) for k, t in enumerate(pr.beta)]
    return dataclasses.replace(pr, alpha=al, beta=be)


def main():
    O.build(force=False)
    pr, sv, theta, theta_true = W.adjoint_config()
    t0 = time.time()
    u0 = I.initial_condition(pr, 0)
    u_obs = O.seq_fine(with_theta(pr, theta_true), u0)[-1]
    L, g_u0, g_th = O.loss_and_gradient(pr, u0, u_obs)
    t1 = time.time()
    rng = np.random.default_rng(2025)
    idx = rng.integers(0, pr.S, 256)
    out = os.path.join(HERE, "adjoint_oracle.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle, 2D adjoint workload; written by tests/golden/make_adjoint_golden.py\n")
        f.write(f"# oracle wall time {t1 - t0:.1f} s (1 core)\n")
        f.write("theta " + " ".join(f"{v:.17e}" for v in theta) + "\n")
        f.write("theta_true " + " ".join(f"{v:.17e}" for v in theta_true) + "\n")
        f.write(f"loss {L:.17e}\n")
        f.write("grad_theta " + " ".join(f"{v:.17e}" for v in g_th) + "\n")
        f.write(f"grad_u0_norm {np.linalg.norm(g_u0):.17e}\n")
        for i in idx:
            f.write(f"grad_u0 {i} {g_u0[i]:.17e}\n")
    print("wrote", out, L, g_th)


if __name__ == "__main__":
    main()
