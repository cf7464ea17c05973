"""Differentiable AMG-PCG solve: x = A(vals)^{-1} b as a torch.autograd.Function.

Forward: A x = b is solved with the preconditioned CG, passing the finest
matrix's values to the solve (a near-by matrix with the hierarchy's pattern,
whose coarse levels stay as built; the library takes them where they differ
from the values in use).  Backward: the adjoint
system A^T lambda = dL/dx is solved with the same hierarchy (A is symmetric),
dL/db = lambda and dL/dvals[k] = -lambda_i x_j for the stored entry (i, j).
All of it runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import mvamg


class AMGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, solver, rtol=1e-10, maxit=1000):
        vals = vals.detach().contiguous()
        x = torch.zeros_like(b)
        info = mvamg.pcg_solve(solver.h, b.detach().contiguous(), x, rtol=rtol, maxit=maxit, A=(None, None, vals))
        if not info.converged:
            raise RuntimeError(f"AMG-PCG did not converge ({info.iterations} iterations, rel. res. {info.rel_res:.2e})")
        ctx.solver, ctx.rtol, ctx.maxit = solver, rtol, maxit
        ctx.save_for_backward(vals, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, x = ctx.saved_tensors
        solver = ctx.solver
        lam = torch.zeros_like(x)
        info = mvamg.adjoint_solve(solver.h, gx.contiguous(), lam, rtol=ctx.rtol, maxit=ctx.maxit,
                                   A=(None, None, vals))
        if not info.converged:
            raise RuntimeError("adjoint AMG-PCG did not converge")
        dvals = torch.empty_like(vals)
        mvamg.grad_coeffs(solver.h, lam, x, dvals)
        return dvals, lam, None, None, None


def amg_solve(vals, b, solver, rtol=1e-10, maxit=1000):
    """x = A(vals)^{-1} b, differentiable in vals and b."""
    return AMGSolve.apply(vals, b, solver, rtol, maxit)
