"""FP64 oracle for the forward models and linearized plug-and-play ADMM.

TEST INFRASTRUCTURE ONLY -- imported by tests/, the smoke check and the bench's
CPU-baseline leg; never by the HIP library.

Super-resolution (Section 4.1): A = decimation by `factor` (keeping samples
factor*I, phase 0) after a blur with kernel b (a separable, normalised Gaussian
in the experiments).  Pixels of the blur support outside the image take the
half-sample symmetric mirror ("symmetric boundary") or wrap around
("periodic").  f(x) = 1/2 ||A x - y||^2 (eq. dataterm) with gradient
A^T (A x - y); the paper prints A^T (y - A x), which is the negative
gradient, so the sign is taken from the data term itself.

Single-photon imaging (Section 4.2): f(x) = sum_i phi(x_i) with
phi(t) = K0 eta t / K - K1 log(1 - exp(-eta t / K)) (eq. obj) and derivative
phi'(t) = (eta/K) (K0 - K1 exp(-eta t/K) / (1 - exp(-eta t/K))) (eq. photongrad),
evaluated at max(t, t_min) so that the logarithm stays finite at t = 0
(the paper leaves the behaviour at the origin open).

Algorithm 1 (Section 2): mu = 1/(alpha + rho); loop
  x <- mu (alpha x + rho (v - u) - grad f(x));  x <- Pi_C(x);
  v <- D(x + u);  u <- u + x - v.
Here D is DSG-NLM with guide x + u (adaptive) for the first k0 iterations and
the weights of iteration k0 afterwards (fixed).  The caller passes alpha
directly; the C library takes gamma = 1/alpha, so that gamma = 1/||A||^2
gives alpha = lambda_max(A^T A), the Lipschitz constant of grad f.
"""
from __future__ import annotations

import math

import numpy as np

from . import dsnlm_ref

__all__ = [
    "gaussian_taps",
    "pad_index",
    "sr_forward",
    "sr_adjoint",
    "sr_dense",
    "power_norm2",
    "spi_counts",
    "spi_phi",
    "spi_grad",
    "spi_ml",
    "ladmm",
    "residual_rms",
]


def gaussian_taps(size: int = 9, sigma: float = 1.0) -> np.ndarray:
    """Sampled Gaussian exp(-k^2 / (2 sigma^2)), k = -(size-1)/2 .. (size-1)/2,
    normalised to sum 1 (one factor of the separable 2-D blur)."""
    k = np.arange(size) - (size - 1) / 2.0
    b = np.exp(-k * k / (2.0 * sigma * sigma))
    return b / b.sum()


def pad_index(n: int, pad: int, boundary: str) -> np.ndarray:
    """Source index in [0, n) of padded positions -pad .. n+pad-1."""
    k = np.arange(-pad, n + pad)
    if boundary == "periodic":
        return np.mod(k, n)
    if boundary != "symmetric":
        raise ValueError(boundary)
    k = np.where(k < 0, -k - 1, k)
    k = np.where(k >= n, 2 * n - 1 - k, k)
    if k.min() < 0 or k.max() >= n:
        raise ValueError("padding wider than the image")
    return k


def sr_forward(x, taps, factor: int, boundary: str = "symmetric") -> np.ndarray:
    """A x: 2-D blur with outer(taps, taps) (direct sum over all size^2 taps),
    then keep every factor-th sample starting at 0."""
    x = np.asarray(x, dtype=np.float64)
    taps = np.asarray(taps, dtype=np.float64)
    n1, n2 = x.shape
    size = taps.size
    r = (size - 1) // 2
    xp = x[pad_index(n1, r, boundary)][:, pad_index(n2, r, boundary)]
    blurred = np.zeros((n1, n2))
    for a in range(size):
        for b in range(size):
            blurred += taps[a] * taps[b] * xp[a:a + n1, b:b + n2]
    return blurred[::factor, ::factor]


def sr_adjoint(res, taps, factor: int, shape, boundary: str = "symmetric") -> np.ndarray:
    """A^T r: zero-insert r onto the HR grid, spread every sample over the
    blur support on the padded grid, then fold the padded margins back onto the
    pixels they were copied from."""
    res = np.asarray(res, dtype=np.float64)
    taps = np.asarray(taps, dtype=np.float64)
    n1, n2 = shape
    size = taps.size
    r = (size - 1) // 2
    up = np.zeros((n1, n2))
    up[::factor, ::factor] = res
    Y = np.zeros((n1 + 2 * r, n2 + 2 * r))
    for a in range(size):
        for b in range(size):
            Y[a:a + n1, b:b + n2] += taps[a] * taps[b] * up
    out = np.zeros((n1, n2))
    ri = pad_index(n1, r, boundary)
    ci = pad_index(n2, r, boundary)
    np.add.at(out, (ri[:, None], ci[None, :]), Y)
    return out


def sr_dense(shape, taps, factor: int, boundary: str = "symmetric") -> np.ndarray:
    """The matrix of A, column by column (tiny shapes only)."""
    n1, n2 = shape
    cols = []
    for k in range(n1 * n2):
        e = np.zeros(n1 * n2)
        e[k] = 1.0
        cols.append(sr_forward(e.reshape(shape), taps, factor, boundary).ravel())
    return np.stack(cols, axis=1)


def power_norm2(apply_AtA, shape, iters: int = 500, seed: int = 0) -> float:
    """Largest eigenvalue of A^T A by power iteration from a seeded start."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply_AtA(v)
        lam = float(np.vdot(v, w))
        v = w / np.linalg.norm(w)
    return lam


def spi_counts(clean, uniforms, eta: float) -> np.ndarray:
    """Number of ones K1 among the K binary measurements of each pixel: a bit is
    1 when its uniform variate falls below the detection probability
    1 - exp(-eta x / K)."""
    clean = np.asarray(clean, dtype=np.float64)
    K = uniforms.shape[-1]
    p1 = -np.expm1(-eta * clean / K)
    return (uniforms.astype(np.float64) < p1[..., None]).sum(-1).astype(np.uint8)


def spi_phi(t, ones, K: int, eta: float, t_min: float = 1e-6) -> np.ndarray:
    """phi(t) of eq. obj, per pixel, at max(t, t_min)."""
    t = np.maximum(np.asarray(t, dtype=np.float64), t_min)
    K1 = np.asarray(ones, dtype=np.float64)
    K0 = K - K1
    return K0 * eta * t / K - K1 * np.log(-np.expm1(-eta * t / K))


def spi_grad(t, ones, K: int, eta: float, t_min: float = 1e-6) -> np.ndarray:
    """phi'(t) of eq. photongrad, per pixel, at max(t, t_min)."""
    t = np.maximum(np.asarray(t, dtype=np.float64), t_min)
    K1 = np.asarray(ones, dtype=np.float64)
    K0 = K - K1
    e = np.exp(-eta * t / K)
    return (eta / K) * (K0 - K1 * e / (-np.expm1(-eta * t / K)))


def spi_ml(ones, K: int, eta: float) -> np.ndarray:
    """Per-pixel maximiser of the likelihood, -(K/eta) log(K0/K) (K0 = 0 is
    mapped to K0 = 1 so the value stays finite)."""
    K1 = np.asarray(ones, dtype=np.float64)
    K0 = np.maximum(K - K1, 1.0)
    return -(K / eta) * np.log(K0 / K)


def residual_rms(a) -> float:
    a = np.asarray(a, dtype=np.float64)
    return float(np.sqrt(np.mean(a * a)))


def ladmm(x0, grad_f, *, alpha: float, rho: float, S: int, P: int, h: float,
          iters: int, freeze_after: int, lo: float = 0.0, hi: float = 1.0,
          v0=None, u0=None, record=None, fixed_guide=None, denoise=None) -> dict:
    """Algorithm 1 with the DSG-NLM denoiser (FP64).

    x0: initial image (v defaults to x0, u to 0).  grad_f: callable x -> grad f.
    Iterations k = 1..iters; for k <= freeze_after the denoiser weights are
    rebuilt from its own input z_k = x^k + u^(k-1); afterwards the weights of
    iteration freeze_after are reused.  If fixed_guide is given, the weights are
    built once from it and never change.  Returns the final x, v, u, the
    per-iteration residuals (RMS of x - v and of rho (v^k - v^(k-1))) and, if
    `record` is a list, appends (x, v, u, z) after every iteration.
    `denoise(z, guide)` defaults to the shift-loop DSG-NLM route; tests with a
    fixed guide may pass the product with the dense matrix W instead.
    """
    if denoise is None:
        def denoise(zz, gg):
            return dsnlm_ref.dsnlm_shifts(zz, gg, S, P, h)["y"].numpy()
    x = np.asarray(x0, dtype=np.float64).copy()
    v = x.copy() if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    u = np.zeros_like(x) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    if fixed_guide is None and freeze_after < 1:
        raise ValueError("freeze_after must be >= 1 (the first iteration builds the weights)")
    mu = 1.0 / (alpha + rho)
    guide = None if fixed_guide is None else np.asarray(fixed_guide, dtype=np.float64)
    res = []
    for k in range(1, iters + 1):
        x = mu * (alpha * x + rho * (v - u) - grad_f(x))
        x = np.clip(x, lo, hi)
        z = x + u
        if fixed_guide is None and k <= freeze_after:
            guide = z.copy()
        v_new = denoise(z, guide)
        dual = rho * (v_new - v)
        v = v_new
        u = u + x - v
        res.append((residual_rms(x - v), residual_rms(dual)))
        if record is not None:
            record.append((x.copy(), v.copy(), u.copy(), z.copy()))
    return dict(x=x, v=v, u=u, residuals=np.asarray(res), guide=guide)


# ---------------------------------------------------------------------------
# Standard plug-and-play ADMM with the inversion solved by conjugate gradients
# (the comparator of Fig. 2; symmetric boundary, where no fast exact
# inversion exists).
# ---------------------------------------------------------------------------
def cg(apply_M, b, x0, iters: int):
    """`iters` conjugate-gradient steps for M x = b (M symmetric positive
    definite, given as a function), started at x0."""
    x = np.asarray(x0, dtype=np.float64).copy()
    r = b - apply_M(x)
    p = r.copy()
    rr = float(np.sum(r * r))
    for _ in range(iters):
        if rr == 0.0:
            break
        q = apply_M(p)
        a = rr / float(np.sum(p * q))
        x = x + a * p
        r = r - a * q
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def admm_cg(x0, y, taps, factor: int, *, rho: float, S: int, P: int, h: float, iters: int,
            freeze_after: int, cg_iters: int, boundary: str = "symmetric", v0=None, u0=None,
            record=None, fixed_guide=None, denoise=None) -> dict:
    """Standard PnP-ADMM for super-resolution: the inversion step is the exact
    minimiser of 1/2||A x - y||^2 + rho/2 ||x - (v - u)||^2, i.e. the solution
    of (A^T A + rho I) x = A^T y + rho (v - u), approximated by `cg_iters`
    conjugate-gradient steps warm-started at the current x (no box
    projection); then v = D(x + u) and u <- u + x - v as in Algorithm 1.
    `record` / `fixed_guide` / `denoise` as in ladmm()."""
    if denoise is None:
        def denoise(zz, gg):
            return dsnlm_ref.dsnlm_shifts(zz, gg, S, P, h)["y"].numpy()
    x = np.asarray(x0, dtype=np.float64).copy()
    v = x.copy() if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    u = np.zeros_like(x) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    shape = x.shape
    Aty = sr_adjoint(np.asarray(y, dtype=np.float64), taps, factor, shape, boundary)

    def apply_M(p):
        return sr_adjoint(sr_forward(p, taps, factor, boundary), taps, factor, shape, boundary) + rho * p

    guide = None if fixed_guide is None else np.asarray(fixed_guide, dtype=np.float64)
    res = []
    for k in range(1, iters + 1):
        x = cg(apply_M, Aty + rho * (v - u), x, cg_iters)
        z = x + u
        if fixed_guide is None and k <= freeze_after:
            guide = z.copy()
        v_new = denoise(z, guide)
        dual = rho * (v_new - v)
        v = v_new
        u = u + x - v
        res.append((residual_rms(x - v), residual_rms(dual)))
        if record is not None:
            record.append((x.copy(), v.copy(), u.copy(), z.copy()))
    return dict(x=x, v=v, u=u, residuals=np.asarray(res), guide=guide)
