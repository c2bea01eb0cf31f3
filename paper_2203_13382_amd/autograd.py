"""``torch.autograd.Function`` over the MGRIT forward solve and the discrete
adjoint of the HIP library: u_nt = Phi(u0, theta), where theta are the
coefficients of the wave-speed terms (the alpha terms, then the beta terms).

Forward keeps only the C-point checkpoints (slm_solve_cpoints); backward runs
slm_adjoint, which solves the adjoint system by MGRIT in reverse time and
recomputes the F-points from the checkpoints while accumulating dL/dtheta.
"""
from __future__ import annotations

import dataclasses

import torch

from .plan import Plan
from . import inputs as I


def with_theta(problem, theta):
    """The problem with its term coefficients replaced by ``theta``."""
    th = [float(v) for v in theta]
    na = len(problem.alpha)
    alpha = [(th[k],) + tuple(t[1:]) for k, t in enumerate(problem.alpha)]
    beta = [(th[na + k],) + tuple(t[1:]) for k, t in enumerate(problem.beta or [])] if problem.dim == 2 else []
    return dataclasses.replace(problem, alpha=alpha, beta=beta if problem.dim == 2 else problem.beta)


class SLMGRITFunction(torch.autograd.Function):
    """apply(u0, theta, problem, solver, seed) -> u_nt (FP64, on the GPU).

    A new plan is set up for the given theta on every call (its departure
    points depend on theta).  The C-point initial iterate of the forward
    solve is the seeded U[0,1) iterate of ``inputs.initial_iterate``."""

    @staticmethod
    def forward(ctx, u0, theta, problem, solver, seed=1):
        pr = with_theta(problem, theta.detach().cpu().tolist())
        plan = Plan(pr, solver, "fp64", device=u0.device, adjoint=True).setup()
        m0 = plan.m[0]
        init = I.initial_iterate(pr.nt, pr.S, m0, seed)[::m0].copy()
        c = torch.from_numpy(init).to(u0.device)
        st, _ = plan.solve_cpoints(u0.detach().to(torch.float64), c)
        if st["status"] not in ("converged",):
            raise RuntimeError(f"forward MGRIT did not converge: {st}")
        ctx.plan, ctx.c, ctx.theta_dtype = plan, c, theta.dtype
        ctx.stats = st
        return c[-1].clone()

    @staticmethod
    def backward(ctx, grad_uT):
        g0, gth, st, _ = ctx.plan.adjoint(ctx.c, grad_uT.detach().to(torch.float64).contiguous())
        if st["status"] not in ("converged",):
            raise RuntimeError(f"adjoint MGRIT did not converge: {st}")
        gt = torch.from_numpy(gth).to(dtype=ctx.theta_dtype)
        return g0.to(grad_uT.dtype), gt, None, None, None
