"""torch.autograd.Function wrappers around the library's forward and backward.

DSNLMFunction: y = W(guide, h) x with gradients for x (W is symmetric, so
the input gradient is W ybar), the guide and h, all computed by the HIP
kernels of dsnlm_apply_backward.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api


class DSNLMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, guide: Optional[torch.Tensor], h: torch.Tensor, S: int, P: int):
        x = x.contiguous()
        self_guided = guide is None
        g = x if self_guided else guide.contiguous()
        hval = float(h)
        y, w = api.dsnlm_forward(x, g, S, P, hval, keep=True)
        ctx.w = w
        ctx.self_guided = self_guided
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        (x,) = ctx.saved_tensors
        need_x = ctx.needs_input_grad[0]
        need_g = ctx.needs_input_grad[1] or (ctx.self_guided and need_x)
        need_h = ctx.needs_input_grad[2]
        dx, dg, dh = api.dsnlm_apply_backward(ctx.w, x, gy.contiguous(), need_dx=need_x or need_g,
                                              need_dguide=need_g, need_dh=need_h)
        if ctx.self_guided:
            gx = dx + dg if need_x else None
            gg = None
        else:
            gx = dx if need_x else None
            gg = dg if ctx.needs_input_grad[1] else None
        gh = dh.reshape(()) if need_h else None
        return gx, gg, gh, None, None


def dsnlm(x: torch.Tensor, guide: Optional[torch.Tensor], h, S: int, P: int) -> torch.Tensor:
    """Differentiable DSG-NLM: W(guide, h) x (guide None = self-guided)."""
    if not isinstance(h, torch.Tensor):
        h = torch.tensor(float(h), device=x.device)
    return DSNLMFunction.apply(x, guide, h, S, P)


class UnrolledLADMM(torch.autograd.Function):
    """x_K = Algorithm 1 run for params.iters iterations from x0 (v0 = x0,
    u0 = 0), differentiable in x0, lambda and rho (bandwidth sqrt(lambda/rho),
    params.h must be <= 0).  The forward keeps per-iteration checkpoints of
    (x, v, u, z); the backward recomputes each iteration's weights from them."""

    @staticmethod
    def forward(ctx, x0, lam, rho, op, params):
        if params.h > 0:
            raise ValueError("UnrolledLADMM differentiates the coupled bandwidth; set params.h <= 0")
        p = api.LadmmParams(**{**params.__dict__, "lam": float(lam), "rho": float(rho)})
        n1, n2 = x0.shape
        x0 = x0.contiguous()
        x, v, u = x0.clone(), x0.clone(), torch.zeros_like(x0)
        ck = torch.empty((p.iters, 4, n1, n2), dtype=torch.float32, device=x0.device)
        api.ladmm_solve(op, p, x, v, u, checkpoints=ck)
        ctx.save_for_backward(x0, ck)
        ctx.op, ctx.p = op, p
        return x

    @staticmethod
    def backward(ctx, gx):
        x0, ck = ctx.saved_tensors
        p = ctx.p
        xb = gx.contiguous().clone()
        vb = torch.zeros_like(xb)
        ub = torch.zeros_like(xb)
        zeros = torch.zeros_like(x0)
        gx0 = torch.empty_like(x0)
        # the library returns the initial image's adjoint (v0 = x0) and dL/dlambda,
        # dL/drho through the coupled bandwidth
        dp = api.ladmm_solve_backward(ctx.op, p, x0, x0, zeros, ck, xb, vb, ub, dinit=gx0)
        return gx0, dp[2], dp[3], None, None


def unrolled_ladmm(x0, lam, rho, op, params):
    lam = lam if isinstance(lam, torch.Tensor) else torch.tensor(float(lam), device=x0.device)
    rho = rho if isinstance(rho, torch.Tensor) else torch.tensor(float(rho), device=x0.device)
    return UnrolledLADMM.apply(x0, lam, rho, op, params)
