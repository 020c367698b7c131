"""Degenerate inputs on the GPU: images of one pixel, one row or one column
and a few pixels, single-image and batched, forward and backward, against
the FP64 oracle.

A 1 x 1 image has no pair besides d = 0, so W = I (omega = 1, c = 1, m = 1)
and y = x exactly; its gradients are x-bar = y-bar, guide-bar = 0 and
h-bar = 0.  Tolerances are those of the other parity tests (2e-5 absolute on
outputs, 1e-4 / 1e-3 relative on gradients).
"""
import numpy as np
import pytest
import torch

from oracle import dsnlm_ref as R
from oracle import grad_ref as G

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _M():
    import paper_1901_06110_amd as M
    return M


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _img(shape, seed):
    return np.random.default_rng(seed).uniform(0, 1, shape).astype(np.float32)


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(a).max())


TINY = [(1, 1, 3, 0), (1, 1, 0, 0), (2, 3, 4, 1), (3, 3, 5, 2), (1, 7, 3, 0), (6, 1, 2, 0)]


@pytest.mark.parametrize("n1,n2,S,P", TINY)
def test_tiny_single_image_forward(n1, n2, S, P):
    M = _M()
    print(f"tiny forward {n1}x{n2} S={S} P={P}", flush=True)
    x, z = _img((n1, n2), 10 + n1 * 7 + n2), _img((n1, n2), 20 + n1 + n2)
    y, w = M.dsnlm_forward(_t(x), _t(z), S, P, 0.1, keep=True)
    torch.cuda.synchronize()
    ref = R.dsnlm_shifts(x, z, S, P, 0.1)
    assert np.abs(y.cpu().numpy() - ref["y"].detach().numpy()).max() <= TOL
    m, _ = w.scalars()
    assert abs(m - float(ref["m"])) <= 1e-5 * float(ref["m"])
    if n1 * n2 == 1:
        assert np.array_equal(y.cpu().numpy(), x)
        assert m == 1.0


def test_tiny_images_batched_forward():
    """A batch mixing 1 x 1, one-row, one-column and small images with a
    larger one (S = 4, P = 0): each image against the oracle with its own h."""
    M = _M()
    shapes = [(1, 1), (1, 9), (9, 1), (2, 3), (40, 70), (1, 1)]
    xs = [_img(s, 40 + k) for k, s in enumerate(shapes)]
    hs = [0.05 + 0.02 * k for k in range(len(shapes))]
    print(f"tiny batched forward {shapes}", flush=True)
    ys = M.dsnlm_forward_batched([(_t(x), _t(x), h) for x, h in zip(xs, hs)], 4, 0)
    torch.cuda.synchronize()
    for k, (x, h, y) in enumerate(zip(xs, hs, ys)):
        ref = R.dsnlm_shifts(x, x, 4, 0, h)["y"].detach().numpy()
        assert np.abs(y.cpu().numpy() - ref).max() <= TOL, k
        m, _, _, _ = M.dsnlm_batched_state(k)
        if x.size == 1:
            assert np.array_equal(y.cpu().numpy(), x) and m == 1.0


# h per case: a bandwidth whose row sums have no near tie at the maximum (the
# gradient of m follows its argmax)
@pytest.mark.parametrize("n1,n2,S,P,h", [(1, 1, 3, 0, 0.1), (2, 3, 4, 1, 0.2), (1, 7, 3, 0, 0.1)])
def test_tiny_single_image_backward(n1, n2, S, P, h):
    M = _M()
    print(f"tiny backward {n1}x{n2} S={S} P={P}", flush=True)
    rng = np.random.default_rng(5 + n1 + n2)
    x, z = _img((n1, n2), 60 + n2), _img((n1, n2), 70 + n1)
    ybar = rng.standard_normal((n1, n2))
    ref = G.autograd_grads(x, z, S, P, h, ybar)
    if n1 * n2 > 1:
        d = np.sort(ref["delta"].ravel())
        assert d[-1] - d[-2] >= 1e-4 * d[-1], "tie in the maximum row sum"
    _, w = M.dsnlm_forward(_t(x), _t(z), S, P, h, keep=True)
    dx, dg, dh = M.dsnlm_apply_backward(w, _t(x), _t(ybar))
    torch.cuda.synchronize()
    assert _rel(dx.cpu().numpy(), ref["dx"]) <= 1e-4
    if n1 * n2 == 1:
        assert np.array_equal(dx.cpu().numpy(), ybar.astype(np.float32))
        assert float(np.abs(dg.cpu().numpy()).max()) == 0.0 and float(dh.cpu()) == 0.0
    else:
        assert _rel(dg.cpu().numpy(), ref["dz"]) <= 1e-3
        assert abs(float(dh.cpu()) - ref["dh"]) <= 1e-3 * abs(ref["dh"])
