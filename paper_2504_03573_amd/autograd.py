"""torch.autograd Functions over the operator and the CG solve.

``SipdgApply``: y = A(lambda, sigma) x.  Backward: dx = A^T gy (the transpose
application), dlambda_e = d(gy^T A x)/dlambda_e and dsigma from the
parameter-gradient kernels.

``SipdgSolve``: u = A(lambda, sigma)^{-1} b by Jacobi-PCG.  The solution u is
kept for the backward pass (the CG state is not differentiated through);
backward solves the adjoint system A w = gu (A is symmetric) and returns
db = w, dlambda = -(w, u)_{Omega_e}, dsigma = -d(w^T A u)/dsigma.

lambda is a float64 device tensor with one entry per element; sigma a
float64 scalar tensor (one penalty scale for every problem of the handle).
"""

from __future__ import annotations

import torch

from .operator import SipdgOperator


def _set_params(op: SipdgOperator, lam: torch.Tensor, sigma: torch.Tensor):
    """Give the handle (lambda, sigma) unless it already holds exactly these:
    the cache key includes the handle's parameter generation, so a direct
    op.set_lambda / op.set_penalty_scale in between is never missed."""
    lam = lam.detach().contiguous()
    if lam.dtype != torch.float64:
        raise TypeError("lambda must be float64")
    key = (lam.data_ptr(), getattr(lam, "_version", 0), float(sigma))
    cached = getattr(op, "_param_key", None)
    if (cached != key or getattr(op, "_param_gen_seen", None) != op.param_generation
            or not torch.equal(getattr(op, "_lam_cache", lam), lam)):
        op.set_lambda(lam)
        op.set_penalty_scale(float(sigma))
        op._lam_cache = lam.clone()
        op._param_key = key
        op._param_gen_seen = op.param_generation


class SipdgApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, lam, sigma, op):
        _set_params(op, lam, sigma)
        y = op.apply(x.detach().contiguous())
        ctx.save_for_backward(x.detach(), lam.detach(), sigma.detach())
        ctx.op = op
        return y

    @staticmethod
    def backward(ctx, gy):
        x, lam, sigma = ctx.saved_tensors
        op = ctx.op
        _set_params(op, lam, sigma)
        gy = gy.contiguous()
        gx = glam = gsig = None
        if ctx.needs_input_grad[0]:
            gx = op.apply_transpose(gy)
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            dl, ds = op.param_grad(gy.double() if gy.dtype != torch.float64 else gy,
                                   x.double() if x.dtype != torch.float64 else x)
            glam = dl
            gsig = ds.sum().reshape(sigma.shape)
        return gx, glam, gsig, None


class SipdgSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, lam, sigma, op, opts):
        _set_params(op, lam, sigma)
        u, info = op.cg_solve(b.detach().contiguous(), **opts)
        ctx.save_for_backward(u, lam.detach(), sigma.detach())
        ctx.op = op
        ctx.opts = opts
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, gu):
        u, lam, sigma = ctx.saved_tensors
        op = ctx.op
        _set_params(op, lam, sigma)
        w, _ = op.cg_solve(gu.contiguous().double(), **ctx.opts)
        gb = w if ctx.needs_input_grad[0] else None
        glam = gsig = None
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            dl, ds = op.param_grad(w, u)
            glam = -dl
            gsig = (-ds.sum()).reshape(sigma.shape)
        return gb, glam, gsig, None, None


def apply(op: SipdgOperator, x: torch.Tensor, lam: torch.Tensor, sigma) -> torch.Tensor:
    sigma = sigma if isinstance(sigma, torch.Tensor) else torch.tensor(float(sigma), dtype=torch.float64, device=x.device)
    return SipdgApply.apply(x, lam, sigma, op)


def solve(op: SipdgOperator, b: torch.Tensor, lam: torch.Tensor, sigma, **opts) -> torch.Tensor:
    sigma = sigma if isinstance(sigma, torch.Tensor) else torch.tensor(float(sigma), dtype=torch.float64, device=b.device)
    opts.setdefault("tol", 1e-12)
    return SipdgSolve.apply(b, lam, sigma, op, opts)
