"""Residual tables in the manner of Tables 2 and 3 (Section 4) on synthetic data.

Runs Algorithm 1 for 250 iterations with three denoisers -- plain NLM (eq. NLM,
rebuilt every iteration), A-DSG-NLM (weights rebuilt every iteration) and
F-DSG-NLM (weights frozen after k0 = 15 iterations, the paper's "typically
15") -- on

* super-resolution: a 512 x 512 piecewise-smooth image, 9 x 9 Gaussian blur
  (sigma 1) and 2x decimation with the periodic boundary of Table 2, noise
  0.01, lambda = 1e-2, rho = 1, gamma = 1/||A||^2, bicubic start;
* single-photon imaging: a 256 x 256 image, K = 16 binary frames, gain
  eta = 4 (the configured case, a very weak signal) and eta = 16, lambda =
  1e-2, rho = 1 (bandwidth sqrt(lambda / rho) = 0.1), alpha = eta^2, start at
  the clipped per-pixel maximum-likelihood value.

For each it prints the primal and dual residuals of the last iteration (RMS
of x - v and of rho (v^k - v^(k-1))) and the PSNR against the clean image.
The solver runs in FP32, so residuals stop shrinking near 1e-7 of the image
scale; the paper's double-precision values go lower.  BM3D is not part of
this library.  Usage: python -m paper_1901_06110_amd.residuals
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

from . import api as M  # noqa: E402

ITERS = 250
K0 = 15


def _psnr(x: np.ndarray, clean: np.ndarray) -> float:
    mse = float(np.mean((np.asarray(x, np.float64) - clean) ** 2))
    return 10.0 * math.log10(1.0 / mse)


def _run(op, params: M.LadmmParams, x0: np.ndarray, clean: np.ndarray) -> dict:
    x = torch.as_tensor(x0).cuda().contiguous()
    v = x.clone()
    u = torch.zeros_like(x)
    res = torch.zeros((params.iters, 2), device="cuda")
    M.ladmm_solve(op, params, x, v, u, residuals=res)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    return dict(primal=float(r[-1, 0]), dual=float(r[-1, 1]), psnr=_psnr(x.cpu().numpy(), clean))


def super_resolution(n: int = 512, S: int = 10, P: int = 3) -> dict:
    cfg = synth.config1_inputs(n)
    b = np.exp(-np.arange(-4, 5) ** 2 / 2.0)
    taps = (b / b.sum()).astype(np.float32)
    op = M.SROperator(n1=n, n2=n, taps=taps, factor=2, y=None, boundary=1)
    clean = np.asarray(cfg["clean"], np.float64)
    y = M.ladmm_apply_forward(op, torch.as_tensor(cfg["clean"]).cuda()) + torch.as_tensor(cfg["lr_noise"]).cuda()
    op.y = y
    x0 = synth.bicubic_upsample(y.cpu().numpy(), 2)
    gamma = 1.0 / M.ladmm_operator_norm2(op, 300)
    out = {}
    for name, den, k0 in (("NLM", 1, 1), ("A-DSG-NLM", 0, ITERS), ("F-DSG-NLM", 0, K0)):
        prm = M.LadmmParams(lam=cfg["lam"], rho=cfg["rho"], gamma=gamma, S=S, P=P, h=cfg["h"], iters=ITERS,
                            freeze_after=k0, denoiser=den)
        out[name] = _run(op, prm, x0, clean)
    out["start"] = dict(psnr=_psnr(x0, clean))
    return out


def single_photon(n: int = 256, K: int = 16, eta: float = 4.0, S: int = 7, P: int = 2) -> dict:
    """Tables-3-style run for one sensor gain eta."""
    clean, uni = synth.config4_batch(count=1, n=n, K=K)[0]
    clean = np.asarray(clean, np.float64)
    # the sensor: frame j of pixel i is 1 when uni < 1 - exp(-eta x_i / K)
    p1 = -np.expm1(-eta * clean / K)
    ones = (uni < p1[..., None]).sum(-1).astype(np.uint8)
    k1 = ones.astype(np.float64)
    k0 = K - k1
    x_ml = np.clip(-(K / eta) * np.log(np.where(k0 > 0, k0 / K, 1.0)), 0.0, 1.0).astype(np.float32)
    op = M.SPIOperator(n1=n, n2=n, ones=torch.as_tensor(ones).cuda(), K=K, eta=eta)
    lam, rho = 1e-2, 1.0
    out = {}
    for name, den, kf in (("NLM", 1, 1), ("A-DSG-NLM", 0, ITERS), ("F-DSG-NLM", 0, K0)):
        prm = M.LadmmParams(lam=lam, rho=rho, gamma=1.0 / (eta * eta), S=S, P=P, h=0.0, iters=ITERS,
                            freeze_after=kf, denoiser=den)
        out[name] = _run(op, prm, x_ml, clean)
    out["start"] = dict(psnr=_psnr(x_ml, clean))
    return out


def main() -> None:
    sr = super_resolution()
    print("super-resolution, 512 x 512, periodic blur, 250 iterations", flush=True)
    _table(sr)
    spi = {}
    for eta in (4.0, 16.0):
        spi[f"eta={eta:g}"] = single_photon(eta=eta)
        print(f"single-photon imaging, 256 x 256, K = 16, eta = {eta:g}, 250 iterations", flush=True)
        _table(spi[f"eta={eta:g}"])
    print(json.dumps({"super_resolution": sr, "single_photon": spi}))


def _table(r: dict) -> None:
    names = ("NLM", "A-DSG-NLM", "F-DSG-NLM")
    print("| | " + " | ".join(names) + " |")
    print("|---|" + "---|" * len(names))
    print("| primal | " + " | ".join(f"{r[k]['primal']:.2e}" for k in names) + " |")
    print("| dual | " + " | ".join(f"{r[k]['dual']:.2e}" for k in names) + " |")
    print("| PSNR (dB) | " + " | ".join(f"{r[k]['psnr']:.2f}" for k in names) + " |")
    print(f"(start PSNR {r['start']['psnr']:.2f} dB)", flush=True)


if __name__ == "__main__":
    main()
