"""torch.autograd view of the reduced functional (paper, Section 2).

J(u) = 1/2 (K u - y_d)^T M_y (K u - y_d) + beta/2 u^T M_u u, K = A^{-1} M_yu.
StateSolve's forward is the state solve y = K u and its hand-written backward
is the adjoint solve K^T g; MassQuad's forward is x^T M x and its backward
2 g M x.  Both run in the HIP library.
"""
from __future__ import annotations

import torch


class StateSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, solver):
        ctx.solver = solver
        return solver.state_solve(u)

    @staticmethod
    def backward(ctx, gy):
        return ctx.solver.adjoint_solve(gy.contiguous()), None


class MassQuad(torch.autograd.Function):
    """q_c = x_c^T M x_c per column; which = 0 (M_u) or 1 (M_y)."""

    @staticmethod
    def forward(ctx, x, solver, which):
        ctx.solver, ctx.which = solver, which
        ctx.save_for_backward(x)
        return solver.mass_quad(x, which).to(x.device)

    @staticmethod
    def backward(ctx, gq):
        (x,) = ctx.saved_tensors
        Mx = ctx.solver.mass_apply(x, ctx.which)
        g = gq.reshape(1, -1) if Mx.dim() == 2 else gq.reshape(())
        return 2.0 * g * Mx, None, None


def reduced_functional(u: torch.Tensor, yd: torch.Tensor, solver) -> torch.Tensor:
    """J per column (shape [nb], or a scalar for a vector u)."""
    y = StateSolve.apply(u, solver)
    e = y - yd
    q = 0.5 * MassQuad.apply(e, solver, 1) + (0.5 * solver.beta) * MassQuad.apply(u, solver, 0)
    return q if u.dim() == 2 else q.reshape(())
