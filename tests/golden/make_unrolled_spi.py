"""Write unrolled_spi_48.json: the FP64 oracle's gradients through 30 unrolled
iterations of Algorithm 1 for single-photon imaging (Section 4.2 model,
K = 16 binary frames, eta = 4; DSG-NLM with S = 7, P = 2, weights frozen after
5 iterations, bandwidth sqrt(lambda / rho), lambda = 1e-2, rho = 1, alpha =
eta^2) on a 48 x 48 image of the seeded single-photon inputs, for
L = ||x_30 - x_clean||^2: dL/dlambda, dL/drho, the adjoint of the initial
image at sampled pixels and its norms, and x_30 at the same pixels.

Calls only oracle/ and synth/.  Run from the repository root:
    python tests/golden/make_unrolled_spi.py
"""
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import grad_ref as G  # noqa: E402
from oracle import ladmm_ref as L  # noqa: E402

N, K, ETA, LAM, RHO, S, P, ITERS, K0 = 48, 16, 4.0, 1e-2, 1.0, 7, 2, 30, 5


def main():
    clean, uni = synth.config4_batch(count=1, n=N, K=K)[0]
    ones = L.spi_counts(clean, uni, ETA)
    x0 = np.clip(L.spi_ml(ones, K, ETA), 0, 1).astype(np.float32)
    lt = torch.tensor(LAM, dtype=torch.float64, requires_grad=True)
    rt = torch.tensor(RHO, dtype=torch.float64, requires_grad=True)
    xt0 = torch.tensor(x0.astype(np.float64), requires_grad=True)
    x, _, _ = G.unrolled_ladmm_torch(xt0, lambda v: G.spi_grad_torch(v, ones, K, ETA), alpha=ETA * ETA,
                                     rho=rt, lam=lt, S=S, P=P, iters=ITERS, freeze_after=K0)
    loss = ((x - torch.as_tensor(clean.astype(np.float64))) ** 2).sum()
    loss.backward()
    g0 = xt0.grad.numpy()
    xk = x.detach().numpy()
    rng = np.random.default_rng(48)
    idx = sorted(set(rng.integers(0, N * N, size=40).tolist()))
    out = dict(n=N, K=K, eta=ETA, lam=LAM, rho=RHO, S=S, P=P, iters=ITERS, freeze_after=K0,
               loss=float(loss), dlambda=float(lt.grad), drho=float(rt.grad),
               dx0_norm2=float(np.sqrt((g0 ** 2).sum())), dx0_maxabs=float(np.abs(g0).max()),
               pixels=idx, dx0=[float(g0.ravel()[i]) for i in idx], x_final=[float(xk.ravel()[i]) for i in idx])
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "unrolled_spi_48.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote unrolled_spi_48.json", out["dlambda"], out["drho"])


if __name__ == "__main__":
    main()
