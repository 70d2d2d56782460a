"""Differentiable solves x = A^{-1} b with hand-written backward passes.

For a loss L(x) with A x = b, the adjoint solve A lambda = dL/dx (A is
symmetric) gives dL/db = lambda and dL/dA_ij = -lambda_i x_j on the stored
entries.  ``SparseSolve`` differentiates with respect to the CSR values and
b; ``DiffusionSolve`` with respect to the per-cell log-coefficients theta of
the 7-point diffusion operator, chaining the value gradient through the
assembly (sspcg_diffusion7_theta_grad).  Both solves, the value gradient and
the chain rule run in the HIP library.
"""
from __future__ import annotations

import torch

from . import solver as S


class SparseSolve(torch.autograd.Function):
    """x = A(val)^{-1} b.  apply(val, b, A, opts) with A a Matrix whose
    values are replaced by val; opts are keyword arguments of solver.solve.
    A matrix stored as one triangle accepts only symmetric val (create it
    with full_storage=True to pass others)."""

    @staticmethod
    def forward(ctx, val, b, A, opts):
        A.update_values(val.detach(), tag=("val", val.data_ptr(), val._version))
        x, _ = S.solve(A, b.detach(), **opts)
        ctx.A, ctx.opts = A, opts
        ctx.save_for_backward(val, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        val, x = ctx.saved_tensors
        A = ctx.A
        tag = ("val", val.data_ptr(), val._version)
        if A.values_tag != tag:
            A.update_values(val.detach(), tag=tag)
        lam, _ = S.solve(A, gx.detach().contiguous(), **ctx.opts)
        gval = S.csr_value_grad(A, lam, x) if ctx.needs_input_grad[0] else None
        return gval, lam, None, None


class DiffusionSolve(torch.autograd.Function):
    """x = A(theta)^{-1} b for the 7-point diffusion operator with
    k = exp(theta).  apply(theta, b, A, opts): A is a Matrix with the 7-point
    pattern (its values are overwritten)."""

    @staticmethod
    def forward(ctx, theta, b, A, opts):
        th = theta.detach().contiguous()
        A.update_values(S.diffusion7_assemble(A, th), tag=("theta", th.data_ptr(), theta._version))
        x, _ = S.solve(A, b.detach(), **opts)
        ctx.A, ctx.opts = A, opts
        ctx.save_for_backward(theta, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        theta, x = ctx.saved_tensors
        A = ctx.A
        th = theta.detach().contiguous()
        tag = ("theta", th.data_ptr(), theta._version)
        if A.values_tag != tag:
            A.update_values(S.diffusion7_assemble(A, th), tag=tag)
        lam, _ = S.solve(A, gx.detach().contiguous(), **ctx.opts)
        gtheta = None
        if ctx.needs_input_grad[0]:
            gval = S.csr_value_grad(A, lam, x)
            gtheta = S.diffusion7_theta_grad(A, th, gval)
        return gtheta, lam, None, None
