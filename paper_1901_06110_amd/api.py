"""Python entry points with the same names as the C ABI (include/dsnlm.h).

Arguments are torch CUDA float32 tensors (2-D, contiguous); the functions pass
their device pointers and the current stream to libdsnlm.so and return
without synchronising, exactly like the C calls.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _img(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous 2-D float32 tensor")
    return t


def _p(t: Optional[torch.Tensor]) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None else None)


class Weights:
    """Owner of a dsnlm_weights handle (freed with the object)."""

    def __init__(self, handle: C.c_void_p, n1: int, n2: int, S: int, P: int, h: float):
        self.handle = handle
        self.n1, self.n2, self.S, self.P, self.h = n1, n2, S, P, h

    def scalars(self):
        """(m, argmax) copied to the host (synchronises the stream)."""
        m = C.c_float()
        am = C.c_int()
        _lib.check(_lib.get().dsnlm_weights_scalars(self.handle, C.byref(m), C.byref(am), _stream()))
        return float(m.value), int(am.value)

    def array(self, which: int) -> torch.Tensor:
        """Copy of the handle's per-pixel array (0: c, 1: delta, 2: guide)."""
        ptr = _lib.get().dsnlm_weights_array(self.handle, which)
        if not ptr:
            raise ValueError("bad array index")
        return _wrap_device(ptr, (self.n1, self.n2)).clone()

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                torch.cuda.current_stream().synchronize()
                _lib.get().dsnlm_weights_destroy(h)
            except Exception:  # pragma: no cover - interpreter shutdown
                pass
            self.handle = None


def _wrap_device(ptr: int, shape) -> torch.Tensor:
    """A tensor view of library-owned float32 device memory (no copy)."""
    class _Arr:
        __cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f4",
                                    "data": (int(ptr), False), "version": 2}
    return torch.as_tensor(_Arr(), device="cuda")


def dsnlm_build_weights(guide: torch.Tensor, S: int, P: int, h: float,
                        out: Optional[Weights] = None) -> Weights:
    guide = _img(guide, "guide")
    n1, n2 = guide.shape
    hp = C.c_void_p(out.handle.value if out is not None else None)
    _lib.check(_lib.get().dsnlm_build_weights(_p(guide), n1, n2, S, P, float(h), _stream(), C.byref(hp)))
    if out is not None:
        out.S, out.P, out.h = S, P, h
        return out
    return Weights(hp, n1, n2, S, P, h)


def dsnlm_apply(w: Weights, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
    x = _img(x, "x")
    if y is None:
        y = torch.empty_like(x)
    _lib.check(_lib.get().dsnlm_apply(w.handle, _p(x), _p(y), _stream()))
    return y


def dsnlm_forward(x: torch.Tensor, guide: Optional[torch.Tensor], S: int, P: int, h: float,
                  y: Optional[torch.Tensor] = None, keep: bool = False,
                  weights: Optional[Weights] = None):
    """y = W(guide) x.  With keep=True (or an existing `weights`), returns
    (y, Weights) so the backward can reuse the saved state."""
    x = _img(x, "x")
    guide = x if guide is None else _img(guide, "guide")
    n1, n2 = x.shape
    if y is None:
        y = torch.empty_like(x)
    if keep or weights is not None:
        hp = C.c_void_p(weights.handle.value if weights is not None else None)
        _lib.check(_lib.get().dsnlm_forward(_p(guide), _p(x), _p(y), n1, n2, S, P, float(h),
                                            _stream(), C.byref(hp)))
        if weights is not None:
            weights.S, weights.P, weights.h = S, P, h
            return y, weights
        return y, Weights(hp, n1, n2, S, P, h)
    _lib.check(_lib.get().dsnlm_forward(_p(guide), _p(x), _p(y), n1, n2, S, P, float(h),
                                        _stream(), None))
    return y


def dsnlm_nlm(x: torch.Tensor, guide: Optional[torch.Tensor], S: int, P: int, h: float,
              y: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Plain NLM (eq. NLM): y_s = sum_r k x_r / sum_r k with the kernel of the
    guide's patches (guide = x when None)."""
    x = _img(x, "x")
    guide = x if guide is None else _img(guide, "guide")
    n1, n2 = x.shape
    if y is None:
        y = torch.empty_like(x)
    _lib.check(_lib.get().dsnlm_nlm(_p(guide), _p(x), _p(y), n1, n2, S, P, float(h), _stream(), None))
    return y


def dsnlm_forward_brute(x: torch.Tensor, guide: Optional[torch.Tensor], S: int, P: int, h: float,
                        y: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The brute-force comparator (patch distances summed directly)."""
    x = _img(x, "x")
    guide = x if guide is None else _img(guide, "guide")
    n1, n2 = x.shape
    if y is None:
        y = torch.empty_like(x)
    _lib.check(_lib.get().dsnlm_forward_brute(_p(guide), _p(x), _p(y), n1, n2, S, P, float(h), _stream(), None))
    return y


def dsnlm_apply_backward(w: Weights, x: torch.Tensor, dy: torch.Tensor, need_dx: bool = True,
                         need_dguide: bool = True, need_dh: bool = True):
    x = _img(x, "x")
    dy = _img(dy, "dy")
    dx = torch.empty_like(x) if need_dx else None
    dg = torch.empty_like(x) if need_dguide else None
    dh = torch.empty((1,), dtype=torch.float32, device=x.device) if need_dh else None
    _lib.check(_lib.get().dsnlm_apply_backward(w.handle, _p(x), _p(dy), _p(dx), _p(dg), _p(dh),
                                               _stream()))
    return dx, dg, dh


_LAST_BATCH: list = []


def dsnlm_forward_batched(images: Sequence, S: int, P: int, outs=None):
    """images: sequence of (guide, x, h); returns the list of outputs."""
    n = len(images)
    arr = (_lib.DsnlmImage * max(n, 1))()
    ys, keep = [], []
    for k, (g, x, h) in enumerate(images):
        x = _img(x, "x")
        g = x if g is None else _img(g, "guide")
        keep.append((g, x))
        y = torch.empty_like(x) if outs is None else outs[k]
        ys.append(y)
        arr[k] = _lib.DsnlmImage(g.data_ptr(), x.data_ptr(), y.data_ptr(), x.shape[0], x.shape[1],
                                 float(h))
    _lib.check(_lib.get().dsnlm_forward_batched(arr, n, S, P, _stream()))
    # the library keeps device pointers to these for dsnlm_backward_batched:
    # hold the tensors until the next batched forward
    _LAST_BATCH[:] = keep
    return ys


def dsnlm_batched_state(image: int):
    """(m, argmax, c, delta) of one image of the last dsnlm_forward_batched
    call; c and delta are copies of the library's device arrays.
    Synchronises the stream."""
    shape = tuple(_LAST_BATCH[image][1].shape)
    m = C.c_float()
    am = C.c_int()
    cp = C.c_void_p()
    dp = C.c_void_p()
    _lib.check(_lib.get().dsnlm_batched_state(int(image), C.byref(m), C.byref(am), C.byref(cp), C.byref(dp),
                                              _stream()))
    return (float(m.value), int(am.value), _wrap_device(cp.value, shape).clone(),
            _wrap_device(dp.value, shape).clone())


def dsnlm_backward_batched(dys: Sequence, need_dx: bool = True, need_dguide: bool = True,
                           need_dh: bool = True):
    """Vector-Jacobian products of the last dsnlm_forward_batched call.

    dys: one cotangent per image of that call, same order.  Its inputs must be
    unchanged.  Returns a list of (dx, dguide, dh) per image (None where not
    requested)."""
    n = len(dys)
    arr = (_lib.DsnlmImageGrad * max(n, 1))()
    res = []
    for k, dy in enumerate(dys):
        dy = _img(dy, "dy")
        dx = torch.empty_like(dy) if need_dx else None
        dg = torch.empty_like(dy) if need_dguide else None
        dh = torch.empty((1,), dtype=torch.float32, device=dy.device) if need_dh else None
        res.append((dx, dg, dh))
        arr[k] = _lib.DsnlmImageGrad(dy.data_ptr(), _p(dx).value, _p(dg).value, _p(dh).value)
    _lib.check(_lib.get().dsnlm_backward_batched(arr, n, _stream()))
    return res


# --------------------------------------------------------------------------
# Linearized plug-and-play ADMM
# --------------------------------------------------------------------------
@dataclasses.dataclass
class SROperator:
    """Blur by outer(taps, taps) then keep every factor-th sample."""
    n1: int
    n2: int
    taps: np.ndarray
    factor: int
    y: Optional[torch.Tensor]
    boundary: int = 0  # 0 symmetric, 1 periodic

    def c_struct(self):
        t = np.ascontiguousarray(self.taps, dtype=np.float32)
        self._taps_keep = t  # keep alive while the struct is used
        s = _lib.LadmmOperator()
        s.kind = _lib.LADMM_OP_SR
        s.n1, s.n2 = self.n1, self.n2
        s.taps = t.ctypes.data_as(C.POINTER(C.c_float))
        s.blur_size = t.size
        s.factor = self.factor
        s.boundary = self.boundary
        s.y = self.y.data_ptr() if self.y is not None else None
        return s


@dataclasses.dataclass
class SPIOperator:
    """Single-photon likelihood: ones[i] of K binary measurements are 1."""
    n1: int
    n2: int
    ones: torch.Tensor  # uint8 CUDA tensor (n1, n2)
    K: int
    eta: float
    t_min: float = 1e-6

    def c_struct(self):
        s = _lib.LadmmOperator()
        s.kind = _lib.LADMM_OP_SPI
        s.n1, s.n2 = self.n1, self.n2
        s.ones = self.ones.data_ptr()
        s.K = self.K
        s.eta = self.eta
        s.t_min = self.t_min
        return s


@dataclasses.dataclass
class LadmmParams:
    lam: float
    rho: float
    gamma: float
    S: int
    P: int
    h: float = 0.0
    iters: int = 1
    freeze_after: int = 1
    lo: float = 0.0
    hi: float = 1.0
    denoiser: int = 0  # 0 DSG-NLM, 1 plain NLM (eq. NLM), rebuilt every iteration

    def c_struct(self):
        return _lib.LadmmParams(self.lam, self.rho, self.gamma, self.S, self.P, self.h, self.iters,
                                self.freeze_after, self.lo, self.hi, self.denoiser)


def ladmm_step(op, params: LadmmParams, k: int, weights: Optional[Weights], x, v, u) -> Weights:
    o = op.c_struct()
    p = params.c_struct()
    hp = C.c_void_p(weights.handle.value if weights is not None else None)
    _lib.check(_lib.get().ladmm_step(C.byref(o), C.byref(p), k, C.byref(hp), _p(x), _p(v), _p(u),
                                     _stream()))
    if weights is not None:
        return weights
    h = params.h if params.h > 0 else math.sqrt(params.lam / params.rho)
    return Weights(hp, op.n1, op.n2, params.S, params.P, h)


def admm_cg_solve(op, params: LadmmParams, cg_iters: int, x, v, u,
                  residuals: Optional[torch.Tensor] = None) -> None:
    """Standard PnP-ADMM with the inversion solved by cg_iters CG steps."""
    o = op.c_struct()
    p = params.c_struct()
    _lib.check(_lib.get().admm_cg_solve(C.byref(o), C.byref(p), int(cg_iters), _p(x), _p(v), _p(u),
                                        _p(residuals), _stream()))


def ladmm_solve(op, params: LadmmParams, x, v, u, residuals: Optional[torch.Tensor] = None,
                checkpoints: Optional[torch.Tensor] = None) -> None:
    o = op.c_struct()
    p = params.c_struct()
    _lib.check(_lib.get().ladmm_solve(C.byref(o), C.byref(p), _p(x), _p(v), _p(u), _p(residuals),
                                      _p(checkpoints), _stream()))


def ladmm_apply_forward(op: SROperator, x: torch.Tensor, out: Optional[torch.Tensor] = None):
    f = op.factor
    if out is None:
        out = torch.empty(((op.n1 + f - 1) // f, (op.n2 + f - 1) // f), dtype=torch.float32,
                          device=x.device)
    o = op.c_struct()
    _lib.check(_lib.get().ladmm_apply_forward(C.byref(o), _p(x), _p(out), _stream()))
    return out


def ladmm_gradient(op, x: torch.Tensor, out: Optional[torch.Tensor] = None):
    if out is None:
        out = torch.empty_like(x)
    o = op.c_struct()
    _lib.check(_lib.get().ladmm_gradient(C.byref(o), _p(x), _p(out), _stream()))
    return out


def ladmm_operator_norm2(op: SROperator, iters: int = 200) -> float:
    o = op.c_struct()
    val = C.c_float()
    _lib.check(_lib.get().ladmm_operator_norm2(C.byref(o), iters, C.byref(val), _stream()))
    return float(val.value)


def ladmm_solve_backward(op, params: LadmmParams, x0, v0, u0, checkpoints, xbar, vbar, ubar,
                         dinit: Optional[torch.Tensor] = None):
    """Reverse pass through ladmm_solve's iterations (checkpoints from the
    forward).  xbar/vbar/ubar are updated in place to the adjoints of the
    initial state; dinit (if given) receives xbar + vbar, the adjoint of an
    initial image used as both x0 and v0.  Returns dparams on the device:
    [explicit d/drho, d/dh, dL/dlambda, dL/drho]."""
    o = op.c_struct()
    p = params.c_struct()
    dparams = torch.empty(4, dtype=torch.float32, device=x0.device)
    _lib.check(_lib.get().ladmm_solve_backward(C.byref(o), C.byref(p), _p(x0), _p(v0), _p(u0),
                                               _p(checkpoints), _p(xbar), _p(vbar), _p(ubar), _p(dinit),
                                               _p(dparams), _stream()))
    return dparams
