"""Reverse-mode differentiation of u = A(v)^-1 b through the COO assembly.

``CooSolve.apply(v, b, A)`` assembles the COO values v into the handle A
(whose pattern came from ``coo_preallocate``), solves A u = b with Jacobi-CG
and returns u.  The hand-written backward, for an upstream gradient g =
dL/du:

  * adjoint solve A^T lam = g (CG on the explicit transpose),
  * dL/db = lam,
  * dL/dA on the stored pattern: G_t = -lam_row(t) u_col(t) (SDDMM),
  * dL/dv[k] = G at the entry triplet k feeds, 0 for ignored triplets
    (the backward of the assembly sum).

``element_coefficient_solve`` covers the finite-element case in which the
triplets of element e are stored contiguously (paper Sec. 5, finite-element
usage) and scale with a per-element coefficient exp(theta_e): v = base +
exp(theta_e) w.  Its backward reduces G * w over each element's block in one
kernel and multiplies by exp(theta_e).  All solves and reductions run in
libspx kernels; torch only carries tensors and the autograd graph.
"""
from __future__ import annotations

import torch

from . import spx


def _require(res, what):
    if res.status != spx.OK:
        raise spx.SpxError(res.status, f"{what} did not converge (relres {res.relres:.3e})")


class CooSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, b, A: "spx.Matrix", rtol: float = 1e-12, maxit: int = 100000):
        A.set_values_coo(v.detach().contiguous())
        res = A.cg_solve(b.detach().contiguous(), rtol=rtol, maxit=maxit)
        _require(res, "forward solve")
        ctx.A, ctx.rtol, ctx.maxit = A, rtol, maxit
        ctx.save_for_backward(v.detach(), res.x)
        return res.x

    @staticmethod
    def backward(ctx, grad_u):
        A = ctx.A
        v, u = ctx.saved_tensors
        A.set_values_coo(v)  # the handle may have been reused since the forward
        adj = A.cg_solve_transpose(grad_u.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        _require(adj, "adjoint solve")
        lam = adj.x
        G = A.sddmm(lam, u)
        grad_v = A.coo_gather(G) if ctx.needs_input_grad[0] else None
        grad_b = lam if ctx.needs_input_grad[1] else None
        return grad_v, grad_b, None, None, None


class ElementCoefficientSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, b, A: "spx.Matrix", base, w, block: int, rtol: float = 1e-12,
                maxit: int = 100000):
        k = torch.exp(theta.detach())
        v = base + torch.repeat_interleave(k, block) * w
        A.set_values_coo(v.contiguous())
        res = A.cg_solve(b.detach().contiguous(), rtol=rtol, maxit=maxit)
        _require(res, "forward solve")
        ctx.A, ctx.block, ctx.rtol, ctx.maxit = A, block, rtol, maxit
        ctx.save_for_backward(k, v, w, res.x)
        return res.x

    @staticmethod
    def backward(ctx, grad_u):
        A = ctx.A
        k, v, w, u = ctx.saved_tensors
        A.set_values_coo(v)
        adj = A.cg_solve_transpose(grad_u.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        _require(adj, "adjoint solve")
        lam = adj.x
        G = A.sddmm(lam, u)
        # dL/dtheta_e = exp(theta_e) * sum_{k in e} G[t(k)] w[k]
        grad_theta = A.coo_gather_blocks(G, w, ctx.block) * k
        grad_b = lam if ctx.needs_input_grad[1] else None
        return grad_theta, grad_b, None, None, None, None, None, None


def coo_solve(v, b, A, rtol=1e-12, maxit=100000):
    """u = A(v)^-1 b, differentiable in v and b."""
    return CooSolve.apply(v, b, A, rtol, maxit)


def element_coefficient_solve(theta, b, A, base, w, block, rtol=1e-12, maxit=100000):
    """u = A(theta)^-1 b with v = base + exp(theta_e) w on element-contiguous
    triplets (block triplets per element); differentiable in theta and b."""
    return ElementCoefficientSolve.apply(theta, b, A, base, w, block, rtol, maxit)
