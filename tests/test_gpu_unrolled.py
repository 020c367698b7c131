"""GPU parity of reverse mode through unrolled linearized PnP-ADMM
(single-photon imaging, adaptive then frozen weights, coupled bandwidth
h = sqrt(lambda / rho)) against FP64 autograd of the unrolled oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import grad_ref as G
from oracle import ladmm_ref as L

pytestmark = pytest.mark.gpu


def _M():
    import paper_1901_06110_amd as M
    return M


def _t(a, dtype=np.float32):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _oracle_grads(x0, clean, ones, K, eta, S, P, iters, k0, lam, rho):
    lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    rt = torch.tensor(rho, dtype=torch.float64, requires_grad=True)
    xt0 = torch.tensor(x0.astype(np.float64), requires_grad=True)
    x, _, _ = G.unrolled_ladmm_torch(xt0, lambda v: G.spi_grad_torch(v, ones, K, eta), alpha=float(eta * eta),
                                     rho=rt, lam=lt, S=S, P=P, iters=iters, freeze_after=k0)
    loss = ((x - torch.as_tensor(clean.astype(np.float64))) ** 2).sum()
    loss.backward()
    return float(lt.grad), float(rt.grad), xt0.grad.numpy(), x.detach().numpy()


@pytest.mark.parametrize("n,S,P,iters,k0", [(24, 3, 1, 6, 3), (32, 7, 2, 8, 5)])
def test_unrolled_spi_parameter_gradients(n, S, P, iters, k0):
    M = _M()
    K, eta, lam, rho = 16, 4.0, 1e-2, 1.0
    clean, uni = synth.config4_batch(count=1, n=n, K=K)[0]
    ones = L.spi_counts(clean, uni, eta)
    x0 = np.clip(L.spi_ml(ones, K, eta), 0, 1).astype(np.float32)
    dl, dr, dx0, xK = _oracle_grads(x0, clean, ones, K, eta, S, P, iters, k0, lam, rho)
    op = M.SPIOperator(n1=n, n2=n, ones=_t(ones, np.uint8), K=K, eta=eta)
    prm = M.LadmmParams(lam=lam, rho=rho, gamma=1.0 / (eta * eta), S=S, P=P, h=0.0, iters=iters,
                        freeze_after=k0)
    x0t = _t(x0).requires_grad_(True)
    lt = torch.tensor(lam, device="cuda", requires_grad=True)
    rt = torch.tensor(rho, device="cuda", requires_grad=True)
    print(f"unrolled SPI {n}x{n} S={S} P={P} iters={iters} k0={k0}", flush=True)
    x = M.unrolled_ladmm(x0t, lt, rt, op, prm)
    assert np.abs(x.detach().cpu().numpy() - xK).max() <= 1e-4
    ((x.double() - _t(clean).double()) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert abs(float(lt.grad) - dl) <= 1e-3 * abs(dl)
    assert abs(float(rt.grad) - dr) <= 1e-3 * abs(dr)
    g = x0t.grad.cpu().numpy()
    assert np.abs(g - dx0).max() <= 1e-3 * np.abs(dx0).max()


def test_unrolled_sr_reverse_step_runs_and_is_deterministic():
    """Super-resolution operator: two reverse passes give identical bits."""
    M = _M()
    n = 32
    clean, _ = synth.piecewise_smooth(n, n, 77, 0.0)
    taps = L.gaussian_taps(9, 1.0).astype(np.float32)
    y = L.sr_forward(clean, taps, 2).astype(np.float32)
    op = M.SROperator(n1=n, n2=n, taps=taps, factor=2, y=_t(y))
    prm = M.LadmmParams(lam=1e-2, rho=1.0, gamma=1 / 0.3321609, S=3, P=1, h=0.0, iters=5, freeze_after=2)
    x0 = _t(synth.bicubic_upsample(y, 2))
    outs = []
    for _ in range(2):
        lt = torch.tensor(1e-2, device="cuda", requires_grad=True)
        rt = torch.tensor(1.0, device="cuda", requires_grad=True)
        x = M.unrolled_ladmm(x0, lt, rt, op, prm)
        ((x - _t(clean)) ** 2).sum().backward()
        outs.append((float(lt.grad), float(rt.grad)))
    assert outs[0] == outs[1]
    assert all(np.isfinite(v) for v in outs[0])


def test_unrolled_spi_thirty_iterations_against_stored_oracle():
    """The configuration's unrolled solve (30 iterations, weights frozen after
    5, S = 7, P = 2, K = 16, eta = 4, coupled bandwidth) on a 48 x 48 image:
    dL/dlambda, dL/drho and the initial image's adjoint against the FP64
    oracle's values stored by tests/golden/make_unrolled_spi.py (the oracle
    takes about a minute here, so it is not rerun in the test)."""
    import json
    import os
    M = _M()
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "unrolled_spi_48.json")))
    n, K, eta = ref["n"], ref["K"], ref["eta"]
    clean, uni = synth.config4_batch(count=1, n=n, K=K)[0]
    ones = L.spi_counts(clean, uni, eta)
    x0 = np.clip(L.spi_ml(ones, K, eta), 0, 1).astype(np.float32)
    op = M.SPIOperator(n1=n, n2=n, ones=_t(ones, np.uint8), K=K, eta=eta)
    prm = M.LadmmParams(lam=ref["lam"], rho=ref["rho"], gamma=1.0 / (eta * eta), S=ref["S"], P=ref["P"], h=0.0,
                        iters=ref["iters"], freeze_after=ref["freeze_after"])
    x0t = _t(x0).requires_grad_(True)
    lt = torch.tensor(ref["lam"], device="cuda", requires_grad=True)
    rt = torch.tensor(ref["rho"], device="cuda", requires_grad=True)
    print(f"unrolled SPI {n}x{n} iters={ref['iters']} against the stored oracle", flush=True)
    x = M.unrolled_ladmm(x0t, lt, rt, op, prm)
    ((x.double() - _t(clean).double()) ** 2).sum().backward()
    torch.cuda.synchronize()
    idx = np.asarray(ref["pixels"])
    assert np.abs(x.detach().cpu().numpy().ravel()[idx] - np.asarray(ref["x_final"])).max() <= 1e-4
    assert abs(float(lt.grad) - ref["dlambda"]) <= 1e-3 * abs(ref["dlambda"])
    assert abs(float(rt.grad) - ref["drho"]) <= 1e-3 * abs(ref["drho"])
    g = x0t.grad.cpu().numpy().ravel()
    assert np.abs(g[idx] - np.asarray(ref["dx0"])).max() <= 1e-3 * ref["dx0_maxabs"]
    assert abs(float(np.sqrt((g.astype(np.float64) ** 2).sum())) - ref["dx0_norm2"]) <= 1e-3 * ref["dx0_norm2"]
