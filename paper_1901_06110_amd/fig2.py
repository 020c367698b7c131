"""Fig. 2 on synthetic data: PSNR against time for linearized and standard
plug-and-play ADMM on super-resolution with the symmetric boundary.

The 512 x 512 super-resolution problem of the bench (9 x 9 Gaussian blur,
sigma 1, 2x decimation, noise 0.01, lambda = 1e-2, rho = 1, DSG-NLM with
S = 10, P = 3, weights rebuilt for 5 iterations then frozen), started at the
bicubic image.  Linearized ADMM (Algorithm 1, gamma = 1/||A||^2) against
standard ADMM whose inversion step (A^T A + rho I) x = A^T y + rho (v - u) is
solved by 5 or 20 conjugate-gradient steps.  Each point is a whole solve of
the given number of iterations, timed on the device (inputs resident), and
the PSNR of its final iterate.  Usage: python -m paper_1901_06110_amd.fig2
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


def _psnr(x: np.ndarray, clean: np.ndarray) -> float:
    return 10.0 * math.log10(1.0 / float(np.mean((np.asarray(x, np.float64) - clean) ** 2)))


def main(n: int = 512) -> None:
    cfg = synth.config1_inputs(n)
    b = np.exp(-np.arange(-4, 5) ** 2 / 2.0)
    taps = (b / b.sum()).astype(np.float32)
    op = M.SROperator(n1=n, n2=n, taps=taps, factor=2, y=None, boundary=0)
    clean = np.asarray(cfg["clean"], np.float64)
    y = M.ladmm_apply_forward(op, torch.as_tensor(cfg["clean"]).cuda()) + torch.as_tensor(cfg["lr_noise"]).cuda()
    op.y = y
    x0 = torch.as_tensor(synth.bicubic_upsample(y.cpu().numpy(), 2)).cuda()
    gamma = 1.0 / M.ladmm_operator_norm2(op, 300)
    st = torch.cuda.Stream()

    def solve(kind: str, iters: int, cg: int = 0):
        prm = M.LadmmParams(lam=cfg["lam"], rho=cfg["rho"], gamma=gamma, S=10, P=3, h=cfg["h"], iters=iters,
                            freeze_after=min(cfg["freeze_after"], iters))
        best = None
        for _ in range(2):  # the second run is timed (first-use costs excluded)
            x, v, u = x0.clone(), x0.clone(), torch.zeros_like(x0)
            torch.cuda.synchronize()
            with torch.cuda.stream(st):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                if kind == "linearized":
                    M.ladmm_solve(op, prm, x, v, u)
                else:
                    M.admm_cg_solve(op, prm, cg, x, v, u)
                e1.record(st)
            torch.cuda.synchronize()
            best = (e0.elapsed_time(e1), _psnr(x.cpu().numpy(), clean))
        return best

    rows = {"bicubic_psnr": _psnr(x0.cpu().numpy(), clean)}
    print(f"bicubic start: {rows['bicubic_psnr']:.2f} dB", flush=True)
    for label, kind, cg in (("linearized ADMM", "linearized", 0), ("standard ADMM, CG 5", "cg", 5),
                            ("standard ADMM, CG 20", "cg", 20)):
        pts = []
        for iters in (1, 2, 3, 5, 8, 12, 20, 30, 50):
            ms, ps = solve(kind, iters, cg)
            pts.append(dict(iters=iters, ms=ms, psnr=ps))
            print(f"{label:22s} iters {iters:3d}  {ms:8.2f} ms  PSNR {ps:6.2f} dB", flush=True)
        rows[label] = pts
    print(json.dumps(rows))


if __name__ == "__main__":
    main()
