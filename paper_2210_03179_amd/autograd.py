"""Differentiable SEM Poisson solve: u = A(G)^{-1} B f as a torch.autograd.Function.

Backward is one adjoint solve through the same preconditioned solver (A is
symmetric, so A^T lambda = dL/du is solved with the forward operator) followed by
the library's contraction kernel, which gives
  dL/df = B lambda,
  dL/dG_aa = -(D_a lambda)(D_a u),  dL/dG_ab = -[(D_a lambda)(D_b u) + (D_b lambda)(D_a u)]
per GLL node (G stored as the six unique components rr, rs, rt, ss, st, tt).
"""
from __future__ import annotations

import torch

from .solver import SemSolver


class SemSolveFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, G, solver: SemSolver, rtol: float, maxit: int):
        solver.set_factors(G.detach())
        b = solver.mass_apply(f.detach().contiguous())
        u, info = solver.solve(b, rtol=rtol, maxit=maxit)
        if not info.converged:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver, ctx.rtol, ctx.maxit = solver, rtol, maxit
        ctx.save_for_backward(u, G)
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, grad_u):
        u, G = ctx.saved_tensors
        solver = ctx.solver
        solver.set_factors(G.detach())
        lam, info = solver.solve(grad_u.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        if not info.converged:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        dG, df = solver.adjoint_contract(lam, u, want_dG=ctx.needs_input_grad[1],
                                         want_df=ctx.needs_input_grad[0])
        return df, dG, None, None, None


def sem_solve(f: torch.Tensor, G: torch.Tensor, solver: SemSolver, rtol: float = 1e-13,
              maxit: int = 2000) -> torch.Tensor:
    """u = A(G)^{-1} B f on the solver's mesh; differentiable in f and G."""
    return SemSolveFunction.apply(f, G, solver, rtol, maxit)
