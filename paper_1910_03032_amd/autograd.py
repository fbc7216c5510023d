"""Differentiable Helmholtz solve: u = A(nu)^{-1} b with A = alpha M + beta K(nu).

Backward (adjoint method): with g = dJ/du, lam solves A lam = g (A is symmetric),
then dJ/dnu_q = -lam^T (dA/dnu_q) u, which the library evaluates pointwise per
quadrature point (K is linear in nu through the stored factor of Section 3.1), and
dJ/db = lam.  The forward solution u is kept as the checkpoint; the backward pass
costs one more PCG solve and one gradient kernel.
"""
from __future__ import annotations

import torch

from . import HELMHOLTZ, Operator


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nu_q, b, op: Operator, alpha, beta, rtol, mode):
        op.set_coeffs(alpha, beta, nu_q.detach())
        u, res = op.pcg(b.detach(), op=HELMHOLTZ, rtol=rtol, mode=mode)
        if not res.converged:
            raise RuntimeError(f"forward solve did not converge: {res}")
        ctx.op, ctx.alpha, ctx.beta, ctx.rtol, ctx.mode = op, alpha, beta, rtol, mode
        ctx.save_for_backward(nu_q.detach(), u)
        return u

    @staticmethod
    def backward(ctx, g_u):
        nu_q, u = ctx.saved_tensors
        op = ctx.op
        # the context may have been re-used with other coefficients since the forward pass
        op.set_coeffs(ctx.alpha, ctx.beta, nu_q)
        lam, res = op.pcg(g_u.contiguous(), op=HELMHOLTZ, rtol=ctx.rtol, mode=ctx.mode)
        if not res.converged:
            raise RuntimeError(f"adjoint solve did not converge: {res}")
        g_nu = op.grad_nu(u, lam).reshape(nu_q.shape)
        return g_nu, lam, None, None, None, None, None


def helmholtz_solve(nu_q, b, op: Operator, alpha=1e3, beta=1.0, rtol=1e-12, mode=0):
    """u(nu) = A(nu)^{-1} b, differentiable in nu_q (per quadrature point) and b."""
    return HelmholtzSolve.apply(nu_q, b, op, alpha, beta, rtol, mode)
