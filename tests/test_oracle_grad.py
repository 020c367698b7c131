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
