"""torch.autograd.Function around the LKS forward and the ALKS adjoint.

forward(gamma) runs Step 2-3 of the optimisation procedure (Sec. 2.7) --
the LKS sweep and the objective -- and returns J as a 0-d double tensor.
backward(gJ) runs Steps 4-5 -- the ALKS sweep seeded with gJ (the adjoint is
linear in its seed) and the sensitivity -- and returns gJ * dJ/dgamma.

The gradient is the paper's ALKS sensitivity, a continuous-adjoint
approximation of the exact derivative of the discrete forward map, not the
exact derivative; torch.autograd.gradcheck is therefore not expected to pass
to its default tolerance.
"""
from __future__ import annotations

import torch

from . import lks


class LKSFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, solver: "lks.LKS", adj_steps=None):
        if gamma.dtype != torch.float64 or not gamma.is_cuda:
            raise TypeError("gamma must be a float64 CUDA tensor")
        g = gamma.detach().contiguous()
        solver.forward(g)
        J = solver.objective()
        solver._token = getattr(solver, "_token", 0) + 1
        ctx.solver = solver
        ctx.token = solver._token
        ctx.adj_steps = adj_steps
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        solver = ctx.solver
        if getattr(solver, "_token", None) != ctx.token:
            # the solver ran another forward since: recompute this one
            solver.forward(g)
            solver._token = getattr(solver, "_token", 0) + 1
            ctx.token = solver._token
        out = torch.empty_like(g)
        solver.backward(float(gJ), out, ctx.adj_steps)
        return out, None, None


def objective(gamma, solver, adj_steps=None):
    """J(gamma) with an ALKS backward; see LKSFunction."""
    return LKSFunction.apply(gamma, solver, adj_steps)
