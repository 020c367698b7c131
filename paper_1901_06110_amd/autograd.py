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
