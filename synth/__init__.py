"""Seeded synthetic inputs shared by the FP64 oracle, the GPU tests and the bench.

This module only draws random numbers and shapes them into images; it holds none
of the restoration method's arithmetic (no patch distances, no kernel weights,
no forward operators).  Every array it returns is float32 (or uint8), so the
GPU path and the oracle read bit-identical inputs.

The paper evaluates on natural photographs (a 256x256 image for the timing table
of Section 3, House for super-resolution, a photon-limited scene for single
photon imaging).  Those images are not available, so a piecewise-smooth
generator stands in for all of them:

1. a linear ramp  a*i/n1 + b*j/n2 + c0,  a, b ~ U[-0.25, 0.25], c0 ~ U[0.25, 0.5];
2. twelve shapes, each a rectangle or a disc with probability 1/2 --
   rectangle: sides U[0.05, 0.3]*(n1, n2) at a uniform position;
   disc: radius U[0.03, 0.15]*min(n1, n2) at a uniform centre;
3. each shape adds an intensity U[0, 1] over its support;
4. clip to [0, 1] (the clean image), then add N(0, sigma_n^2) noise, no re-clip.

Seeds: configuration c, image i uses numpy default_rng(1000*c + i).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "piecewise_smooth",
    "config0",
    "config1_inputs",
    "config2_batch",
    "config3_batch",
    "config4_batch",
    "bicubic_upsample",
    "BatchItem",
]


def piecewise_smooth(n1: int, n2: int, seed: int, sigma_n: float):
    """Return (clean, noisy) float32 images of shape (n1, n2).

    The draw order is fixed (ramp, then 12 shapes, then the noise field) so a
    given (n1, n2, seed, sigma_n) always yields the same arrays.
    """
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(-0.25, 0.25, size=2)
    c0 = rng.uniform(0.25, 0.5)
    ii = np.arange(n1, dtype=np.float64)[:, None]
    jj = np.arange(n2, dtype=np.float64)[None, :]
    img = a * ii / n1 + b * jj / n2 + c0 + np.zeros((n1, n2))
    for _ in range(12):
        if rng.uniform() < 0.5:
            hh = rng.uniform(0.05, 0.3) * n1
            ww = rng.uniform(0.05, 0.3) * n2
            r0 = rng.uniform(0.0, max(n1 - hh, 0.0))
            q0 = rng.uniform(0.0, max(n2 - ww, 0.0))
            mask = (ii >= r0) & (ii < r0 + hh) & (jj >= q0) & (jj < q0 + ww)
        else:
            rad = rng.uniform(0.03, 0.15) * min(n1, n2)
            ci = rng.uniform(0.0, n1)
            cj = rng.uniform(0.0, n2)
            mask = (ii - ci) ** 2 + (jj - cj) ** 2 <= rad * rad
        img = img + rng.uniform(0.0, 1.0) * mask
    clean = np.clip(img, 0.0, 1.0)
    noisy = clean + rng.normal(0.0, sigma_n, size=(n1, n2))
    return clean.astype(np.float32), noisy.astype(np.float32)


def config0():
    """64x64 denoising case: search half-width 5, patch half-width 2, h = 0.1.

    Returns a dict with the noisy image (which is also the guide) and the clean one.
    """
    clean, noisy = piecewise_smooth(64, 64, seed=0, sigma_n=0.05)
    return dict(x=noisy, guide=noisy, clean=clean, S=5, P=2, h=0.1)


def config1_inputs(n: int = 512, lr_noise_sigma: float = 0.01):
    """2x super-resolution case on an n x n ground truth.

    Returns the clean HR image and the LR noise field (shape (n/2, n/2)); the
    observation y = A x + noise is formed by whoever owns the operator A.
    Parameters of the restoration follow the configuration: blur 9x9 Gaussian
    sigma 1, factor 2, lambda 1e-2, rho 1, S = 10, P = 3, h = 0.05, 50
    iterations, weights frozen after 5.
    """
    clean, _ = piecewise_smooth(n, n, seed=1000, sigma_n=0.0)
    rng = np.random.default_rng(1000 + 500)
    noise = rng.normal(0.0, lr_noise_sigma, size=(n // 2, n // 2)).astype(np.float32)
    return dict(clean=clean, lr_noise=noise, blur_size=9, blur_sigma=1.0, factor=2,
                lam=1e-2, rho=1.0, S=10, P=3, h=0.05, iters=50, freeze_after=5)


@dataclasses.dataclass
class BatchItem:
    clean: np.ndarray
    noisy: np.ndarray
    sigma_n: float
    h: float


def config2_batch(count: int = 64, sides=(128, 256, 384, 512, 768, 1024)):
    """Batch of images of uneven sizes: side s drawn from `sides`, square with
    probability 1/2 else s/2 x s; sigma_n ~ U[0.02, 0.1]; h = 1.2 sigma_n.

    The shapes and noise levels come from default_rng(2999); image i uses seed
    2000 + i.
    """
    rng = np.random.default_rng(2999)
    items = []
    for i in range(count):
        s = int(rng.choice(np.asarray(sides)))
        square = rng.uniform() < 0.5
        n1, n2 = (s, s) if square else (s // 2, s)
        sig = float(rng.uniform(0.02, 0.1))
        clean, noisy = piecewise_smooth(n1, n2, seed=2000 + i, sigma_n=sig)
        items.append(BatchItem(clean=clean, noisy=noisy, sigma_n=sig, h=1.2 * sig))
    return items


def config3_batch(count: int = 8, n: int = 256):
    """Batch of count images n x n, sigma_n = 0.05 (differentiated denoiser case)."""
    out = []
    for i in range(count):
        clean, noisy = piecewise_smooth(n, n, seed=3000 + i, sigma_n=0.05)
        out.append((clean, noisy))
    return out


def config4_batch(count: int = 16, n: int = 256, K: int = 16):
    """Single-photon case: clean intensities in [0, 1] plus, per pixel, K
    uniform U[0, 1) variates that the sensor model thresholds into binary
    measurements (the thresholding itself belongs to the measurement model).
    Returns a list of (clean, uniforms[n, n, K]) pairs.
    """
    out = []
    for i in range(count):
        clean, _ = piecewise_smooth(n, n, seed=4000 + i, sigma_n=0.0)
        rng = np.random.default_rng(4000 + 500 + i)
        uni = rng.uniform(0.0, 1.0, size=(n, n, K)).astype(np.float32)
        out.append((clean, uni))
    return out


def _keys_cubic(t: np.ndarray, a: float = -0.5) -> np.ndarray:
    """Keys' cubic convolution kernel (a = -0.5)."""
    t = np.abs(t)
    w = np.zeros_like(t)
    m1 = t <= 1
    m2 = (t > 1) & (t < 2)
    w[m1] = (a + 2) * t[m1] ** 3 - (a + 3) * t[m1] ** 2 + 1
    w[m2] = a * t[m2] ** 3 - 5 * a * t[m2] ** 2 + 8 * a * t[m2] - 4 * a
    return w


def bicubic_upsample(lr: np.ndarray, factor: int) -> np.ndarray:
    """Bicubic (Keys, a = -0.5) interpolation of an LR image onto the HR grid
    whose sample factor*I coincides with LR sample I; edge samples are
    replicated.  Used only to initialise the super-resolution iterations.
    """
    lr = np.asarray(lr, dtype=np.float64)
    m1, m2 = lr.shape

    def axis_matrix(m: int) -> np.ndarray:
        n = m * factor
        pos = np.arange(n) / factor
        base = np.floor(pos).astype(int)
        mat = np.zeros((n, m))
        for off in (-1, 0, 1, 2):
            idx = base + off
            w = _keys_cubic(pos - idx)
            np.add.at(mat, (np.arange(n), np.clip(idx, 0, m - 1)), w)
        return mat

    up = axis_matrix(m1) @ lr @ axis_matrix(m2).T
    return up.astype(np.float32)
