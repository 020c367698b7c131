"""Reference gradients for the differentiated denoiser (FP64).

TEST INFRASTRUCTURE ONLY -- imported by tests/ and the smoke check; never by
the HIP library.

The paper does not differentiate its denoiser; the gradients here follow from
the forward definition (Section 3, eqs. NLM and S1-S3) by the chain rule.
Two independent references are provided:

* `autograd_grads` -- torch CPU float64 autograd through the band-by-band
  route of steps S1-S3 (dsnlm_ref.dsnlm_shifts); the derivative of the maximum row
  sum is routed to the first maximal pixel;
* `central_fd`     -- central finite differences of the same FP64 forward.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dsnlm_ref

__all__ = ["autograd_grads", "central_fd", "loss_value"]


def loss_value(x, z, S, P, h, target=None, ybar=None) -> float:
    """L = ||W(z, h) x - target||^2 if target is given, else <W(z, h) x, ybar>."""
    y = dsnlm_ref.dsnlm_shifts(x, z, S, P, h)["y"]
    if target is not None:
        t = torch.as_tensor(np.asarray(target, dtype=np.float64))
        return float(((y - t) ** 2).sum())
    return float((y * torch.as_tensor(np.asarray(ybar, dtype=np.float64))).sum())


def autograd_grads(x, z, S, P, h, ybar) -> dict:
    """Gradients of <W(z, h) x, ybar> with respect to x, z and h (FP64)."""
    xt = torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=True)
    zt = torch.tensor(np.asarray(z, dtype=np.float64), requires_grad=True)
    ht = torch.tensor(float(h), dtype=torch.float64, requires_grad=True)
    out = dsnlm_ref.dsnlm_shifts(xt, zt, S, P, ht)
    yb = torch.as_tensor(np.asarray(ybar, dtype=np.float64))
    (out["y"] * yb).sum().backward()
    return dict(dx=xt.grad.numpy(), dz=zt.grad.numpy(), dh=float(ht.grad),
                y=out["y"].detach().numpy(), m=float(out["m"]), argmax=out["argmax"],
                delta=out["delta"].detach().numpy())


def central_fd(fun, arr, idx_list, step: float = 1e-3) -> np.ndarray:
    """Central differences (fun(a + step e_k) - fun(a - step e_k)) / (2 step)
    at the flat indices idx_list of arr (or of the scalar, if arr is a float)."""
    if np.isscalar(arr):
        return np.asarray([(fun(arr + step) - fun(arr - step)) / (2 * step)])
    a = np.asarray(arr, dtype=np.float64)
    out = []
    for k in idx_list:
        ap = a.copy().ravel()
        am = a.copy().ravel()
        ap[k] += step
        am[k] -= step
        out.append((fun(ap.reshape(a.shape)) - fun(am.reshape(a.shape))) / (2 * step))
    return np.asarray(out)


# ---------------------------------------------------------------------------
# Unrolled Algorithm 1 in torch FP64 (differentiable in lambda, rho, h)
# ---------------------------------------------------------------------------
def _box(q, lo, hi):
    """Pi_C with derivative 1 strictly inside the box and 0 elsewhere."""
    inside = (q > lo) & (q < hi)
    return torch.where(inside, q, torch.clamp(q, lo, hi).detach())


def spi_grad_torch(t, ones, K, eta, t_min=1e-6):
    """phi'(t) of the single-photon likelihood at max(t, t_min) (derivative of
    the max taken as 1 above t_min and 0 below)."""
    t = torch.where(t > t_min, t, torch.full_like(t, t_min))
    K1 = torch.as_tensor(np.asarray(ones, dtype=np.float64))
    K0 = K - K1
    a = eta * t / K
    return (eta / K) * (K0 - K1 * torch.exp(-a) / (-torch.expm1(-a)))


def unrolled_ladmm_torch(x0, grad_f, *, alpha, rho, lam, S, P, iters, freeze_after, lo=0.0, hi=1.0,
                         h=None, v0=None, u0=None):
    """Algorithm 1 unrolled in torch FP64.  rho, lam (and h, if given) may be
    tensors requiring grad; without h the bandwidth is sqrt(lam / rho).
    Returns the final (x, v, u)."""
    x = x0
    v = x0 if v0 is None else v0
    u = torch.zeros_like(x0) if u0 is None else u0
    hh = torch.sqrt(lam / rho) if h is None else h
    mu = 1.0 / (alpha + rho)
    guide = None
    for k in range(1, iters + 1):
        q = mu * (alpha * x + rho * (v - u) - grad_f(x))
        x = _box(q, lo, hi)
        z = x + u
        if k <= freeze_after:
            guide = z
        v = dsnlm_ref.dsnlm_shifts(z, guide, S, P, hh)["y"]
        u = u + x - v
    return x, v, u
