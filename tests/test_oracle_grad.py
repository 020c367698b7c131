"""CPU pins for the FP64 reference gradients (no GPU).

The autograd reference is checked against central finite differences of the
forward, and its input gradient against the product with W itself (W is
symmetric, so the adjoint of x -> W x is W).
"""
import numpy as np

import synth
from oracle import dsnlm_ref as R
from oracle import grad_ref as G


def _case(n1=9, n2=8, seed=51):
    _, z = synth.piecewise_smooth(n1, n2, seed, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, seed + 1, 0.05)
    ybar = np.random.default_rng(seed).standard_normal((n1, n2))
    return x.astype(np.float64), z.astype(np.float64), ybar


def test_input_gradient_is_W_times_cotangent():
    x, z, ybar = _case()
    S, P, h = 2, 1, 0.1
    g = G.autograd_grads(x, z, S, P, h, ybar)
    W = R.dense_weights(z, S, P, h)["W"]
    assert np.abs(g["dx"].ravel() - W.T @ ybar.ravel()).max() <= 1e-13
    assert np.abs(g["dx"].ravel() - W @ ybar.ravel()).max() <= 1e-13


def test_guide_and_bandwidth_gradients_vs_central_fd():
    x, z, ybar = _case()
    S, P, h = 2, 1, 0.1
    g = G.autograd_grads(x, z, S, P, h, ybar)
    # keep away from a tie in the maximum row sum (derivative of max)
    d = np.sort(g["delta"].ravel())
    assert d[-1] - d[-2] >= 1e-4 * d[-1]
    idx = [0, 7, 20, 41, 55, 71]
    fd = G.central_fd(lambda zz: G.loss_value(x, zz, S, P, h, ybar=ybar), z, idx, step=1e-5)
    an = g["dz"].ravel()[idx]
    assert np.abs(fd - an).max() <= 1e-6 * max(1.0, np.abs(an).max())
    fdh = G.central_fd(lambda hh: G.loss_value(x, z, S, P, hh, ybar=ybar), h, None, step=1e-6)[0]
    assert abs(fdh - g["dh"]) <= 1e-6 * max(1.0, abs(g["dh"]))


def _spi_case(n=10, K=16, eta=4.0, seed=5):
    from oracle import ladmm_ref as L
    clean, uni = synth.config4_batch(count=1, n=n, K=K)[0]
    ones = L.spi_counts(clean, uni, eta)
    x0 = np.clip(L.spi_ml(ones, K, eta), 0, 1)
    return clean.astype(np.float64), ones, x0


def test_unrolled_torch_matches_numpy_algorithm1():
    """The differentiable unrolled LADMM reproduces the numpy Algorithm 1."""
    import torch
    from oracle import ladmm_ref as L
    K, eta, S, P = 16, 4.0, 2, 1
    clean, ones, x0 = _spi_case()
    lam, rho = 1e-2, 1.0
    h = np.sqrt(lam / rho)
    out = L.ladmm(x0, lambda v: L.spi_grad(v, ones, K, eta), alpha=16.0, rho=rho, S=S, P=P, h=h,
                  iters=4, freeze_after=2)
    xt, vt, ut = G.unrolled_ladmm_torch(
        torch.as_tensor(x0), lambda v: G.spi_grad_torch(v, ones, K, eta), alpha=16.0,
        rho=torch.tensor(rho, dtype=torch.float64), lam=torch.tensor(lam, dtype=torch.float64),
        S=S, P=P, iters=4, freeze_after=2)
    assert np.abs(xt.numpy() - out["x"]).max() <= 1e-13
    assert np.abs(vt.numpy() - out["v"]).max() <= 1e-13
    assert np.abs(ut.numpy() - out["u"]).max() <= 1e-13


def test_unrolled_parameter_gradients_vs_central_fd():
    import torch
    K, eta, S, P = 16, 4.0, 2, 1
    clean, ones, x0 = _spi_case()

    def loss(lam, rho):
        lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
        rt = torch.tensor(rho, dtype=torch.float64, requires_grad=True)
        x, _, _ = G.unrolled_ladmm_torch(torch.as_tensor(x0), lambda v: G.spi_grad_torch(v, ones, K, eta),
                                         alpha=16.0, rho=rt, lam=lt, S=S, P=P, iters=4, freeze_after=2)
        val = ((x - torch.as_tensor(clean)) ** 2).sum()
        return val, lt, rt

    val, lt, rt = loss(1e-2, 1.0)
    val.backward()
    step = 1e-6
    fdl = (float(loss(1e-2 + step, 1.0)[0]) - float(loss(1e-2 - step, 1.0)[0])) / (2 * step)
    fdr = (float(loss(1e-2, 1.0 + step)[0]) - float(loss(1e-2, 1.0 - step)[0])) / (2 * step)
    assert abs(float(lt.grad) - fdl) <= 1e-5 * max(1.0, abs(fdl))
    assert abs(float(rt.grad) - fdr) <= 1e-5 * max(1.0, abs(fdr))
