"""torch.autograd wrappers of the DDELM-NN solve and evaluation.

Both maps are linear in their tensor inputs, so the backward of each is
the library's adjoint call: ddelm_solve_adjoint for the solve (the
transposed interface system, one more CG with the stored factors) and
ddelm_evaluate_adjoint for the evaluation.  Gradients flow to the data
(f at the interior points, g at the boundary points) and to the
last-layer coefficients; the hidden parameters and the points are
constants of the method (sec. 2.2) and get no gradient.
"""
from __future__ import annotations

import torch

from .solver import DDELMSolver


class DDSolve(torch.autograd.Function):
    """coef = solve(f_I, g_B) with coef_bar -> (f_I_bar, g_B_bar) by the adjoint."""

    @staticmethod
    def forward(ctx, solver: DDELMSolver, f_I: torch.Tensor, g_B: torch.Tensor):
        ctx.solver = solver
        ctx.batched = f_I.ndim == 3
        out = solver.solve(f_I.detach(), g_B.detach(), want_mu=False)
        ctx.stats = out["stats"]
        return out["coef"] if ctx.batched else out["coef"][0]

    @staticmethod
    def backward(ctx, coef_bar):
        cb = coef_bar if ctx.batched else coef_bar[None]
        adj = ctx.solver.solve_adjoint(cb)
        fI, gB = adj["f_I_bar"], adj["g_B_bar"]
        if not ctx.batched:
            fI, gB = fI[0], gB[0]
        return None, fI, gB


class DDEvaluate(torch.autograd.Function):
    """u = evaluate(coef, x) with u_bar -> coef_bar by the evaluation adjoint."""

    @staticmethod
    def forward(ctx, solver: DDELMSolver, coef: torch.Tensor, x: torch.Tensor):
        ctx.solver = solver
        ctx.batched = coef.ndim == 3
        ctx.save_for_backward(x)
        c = coef.detach() if ctx.batched else coef.detach()[None]
        u = solver.evaluate(c, x)
        return u if ctx.batched else u[0]

    @staticmethod
    def backward(ctx, u_bar):
        (x,) = ctx.saved_tensors
        ub = u_bar if ctx.batched else u_bar[None]
        cb = ctx.solver.evaluate_adjoint(x, ub.contiguous())
        return None, (cb if ctx.batched else cb[0]), None


def solve(solver: DDELMSolver, f_I: torch.Tensor, g_B: torch.Tensor) -> torch.Tensor:
    """Differentiable coefficients c(f_I, g_B)."""
    return DDSolve.apply(solver, f_I, g_B)


def evaluate(solver: DDELMSolver, coef: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Differentiable u(x) for the coefficients coef."""
    return DDEvaluate.apply(solver, coef, x)
