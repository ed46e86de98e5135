"""torch.autograd.Function around the s-step enlarged CG solve.

For x = A^{-1} b with A symmetric positive definite and a scalar loss L(x):
  lambda = A^{-1} dL/dx          (adjoint solve; A^t = A, same solver)
  dL/db  = lambda
  dL/dA_ij = -lambda_i x_j       on the stored nonzeros (SDDMM kernel)
Both solves and the SDDMM run in the library's HIP kernels.
"""
from __future__ import annotations

import torch


class ECGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, solver, tol, maxit):
        x, info = solver.solve(b, tol=tol, maxit=maxit)
        if info.status != 0:
            raise RuntimeError(f"forward solve did not converge (status {info.status})")
        ctx.solver, ctx.tol, ctx.maxit = solver, tol, maxit
        ctx.save_for_backward(x)
        ctx.forward_info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam, info = ctx.solver.solve(gx.detach().contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        if info.status != 0:
            raise RuntimeError(f"adjoint solve did not converge (status {info.status})")
        gvals = ctx.solver.sddmm(lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gvals, gb, None, None, None


def solve_with_grad(rowptr, colind, vals: torch.Tensor, partition, t: int, s: int,
                    b: torch.Tensor, *, tol: float = 1e-8, maxit: int = 10000, **opts):
    """x = A(vals)^{-1} b, differentiable with respect to vals and b."""
    from . import Solver
    solver = Solver(rowptr, colind, vals.detach(), partition, t, s, **opts)
    return ECGSolve.apply(vals, b, solver, tol, maxit)
