"""GPU parity of the DSG-NLM forward path against the FP64 oracle.

Tolerance: max-abs 2e-5 on [0, 1] images (outputs of the FP32 kernels vs the
FP64 shift-loop oracle on the same float32 inputs).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dsnlm_ref as R

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _gpu():
    import paper_1901_06110_amd as M
    return M


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _oracle(x, z, S, P, h):
    out = R.dsnlm_shifts(x, z, S, P, h)
    return (out["y"].numpy(), float(out["m"]), out["argmax"], out["omega"].numpy(),
            out["delta"].numpy())


CASES = [
    # (n1, n2, S, P, h): several tiles, ragged tails, S >= size, P >= S, 1-wide
    (64, 64, 5, 2, 0.1),
    (37, 131, 3, 1, 0.08),
    (100, 70, 7, 3, 0.05),
    (65, 129, 10, 3, 0.05),
    (5, 9, 6, 2, 0.1),
    (1, 40, 2, 0, 0.1),
    (40, 1, 2, 0, 0.1),
    (33, 65, 2, 4, 0.2),
    (70, 33, 0, 2, 0.1),
    (12, 200, 4, 5, 0.15),
    (256, 256, 10, 3, 0.024),   # smallest bandwidth of the batched workload
    (96, 160, 8, 5, 0.03),
]


@pytest.mark.parametrize("n1,n2,S,P,h", CASES)
def test_forward_matches_oracle(n1, n2, S, P, h):
    M = _gpu()
    print(f"forward case {n1}x{n2} S={S} P={P} h={h}", flush=True)
    _, z = synth.piecewise_smooth(n1, n2, 100 + n1 + n2, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, 200 + n1 + n2, 0.05)
    y, w = M.dsnlm_forward(_t(x), _t(z), S, P, h, keep=True)
    torch.cuda.synchronize()
    yo, mo, amo, om, dl = _oracle(x, z, S, P, h)
    err = np.abs(y.cpu().numpy() - yo).max()
    assert err <= TOL, err
    m, am = w.scalars()
    assert abs(m - mo) <= 1e-5 * mo
    d = np.sort(dl.ravel())
    if d.size == 1 or d[-1] - d[-2] > 1e-4 * d[-1]:
        assert am == amo
    c = w.array(0).cpu().numpy()
    assert np.abs(c / om ** -0.5 - 1).max() <= 2e-5
    assert np.abs(w.array(1).cpu().numpy() - dl).max() <= 2e-5


def test_config0_and_self_guided():
    M = _gpu()
    cfg = synth.config0()
    x = _t(cfg["x"])
    y = M.dsnlm_forward(x, None, cfg["S"], cfg["P"], cfg["h"])
    yo = _oracle(cfg["x"], cfg["guide"], cfg["S"], cfg["P"], cfg["h"])[0]
    assert np.abs(y.cpu().numpy() - yo).max() <= TOL


def test_build_then_apply_equals_fused_forward():
    """Building the weights and applying them (three sweeps) gives exactly the
    fused forward (two sweeps): same accumulation order per pixel."""
    M = _gpu()
    _, z = synth.piecewise_smooth(90, 77, 7, 0.05)
    _, x = synth.piecewise_smooth(90, 77, 8, 0.05)
    zt, xt = _t(z), _t(x)
    w = M.dsnlm_build_weights(zt, 6, 2, 0.07)
    y1 = M.dsnlm_apply(w, xt)
    y2 = M.dsnlm_forward(xt, zt, 6, 2, 0.07)
    assert torch.equal(y1, y2)
    # frozen weights: the guide buffer may change after the build
    zt.add_(0.3)
    y3 = M.dsnlm_apply(w, xt)
    assert torch.equal(y1, y3)
    # rebuilding in place re-uses the handle
    w2 = M.dsnlm_build_weights(_t(z), 6, 2, 0.07, out=w)
    assert w2 is w
    assert torch.equal(M.dsnlm_apply(w, xt), y1)


def test_invariants_on_gpu():
    """Symmetry <W x, v> = <x, W v>, constants kept, mean preserved, output
    inside [min x, max x], on the GPU output itself."""
    M = _gpu()
    _, z = synth.piecewise_smooth(160, 96, 17, 0.05)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (160, 96)).astype(np.float32)
    v = rng.uniform(0, 1, (160, 96)).astype(np.float32)
    w = M.dsnlm_build_weights(_t(z), 10, 3, 0.05)
    wx = M.dsnlm_apply(w, _t(x)).double().cpu().numpy()
    wv = M.dsnlm_apply(w, _t(v)).double().cpu().numpy()
    a = float((wx * v).sum())
    b = float((x.astype(np.float64) * wv).sum())
    assert abs(a - b) <= 1e-5 * abs(a)
    one = M.dsnlm_apply(w, torch.full((160, 96), 0.42, device="cuda")).cpu().numpy()
    assert np.abs(one - np.float32(0.42)).max() <= 1e-6
    assert abs(wx.sum() - x.astype(np.float64).sum()) <= 1e-5 * x.size
    assert wx.min() >= x.min() - 1e-6 and wx.max() <= x.max() + 1e-6


def test_vanishing_bandwidth_identity_on_gpu():
    M = _gpu()
    rng = np.random.default_rng(9)
    z = rng.uniform(0, 1, (50, 70)).astype(np.float32)
    x = rng.uniform(0, 1, (50, 70)).astype(np.float32)
    y = M.dsnlm_forward(_t(x), _t(z), 4, 1, 1e-6)
    assert np.array_equal(y.cpu().numpy(), x)


def test_full_size_512_matches_oracle():
    """The 512x512 configuration at S = 10, P = 3 in the launch shape the
    bench times, compared with the oracle over every pixel."""
    M = _gpu()
    cfg = synth.config1_inputs(512)
    _, x = synth.piecewise_smooth(512, 512, 1001, 0.05)
    print("full-size 512x512 S=10 P=3", flush=True)
    y = M.dsnlm_forward(_t(x), None, 10, 3, cfg["h"])
    yo = _oracle(x, x, 10, 3, cfg["h"])[0]
    assert np.abs(y.cpu().numpy() - yo).max() <= TOL


def test_batched_equals_per_image_and_oracle():
    """One launch per sweep over uneven images gives the per-image result (same
    tiles; a small single image splits each tile's shifts over several blocks,
    so the two differ by summation order only), and each image matches the
    oracle with its own m and h."""
    M = _gpu()
    shapes = [(64, 128), (33, 17), (128, 64), (7, 200), (96, 96), (3, 50)]
    items = []
    for k, (a, b) in enumerate(shapes):
        _, x = synth.piecewise_smooth(a, b, 700 + k, 0.03 + 0.01 * k)
        items.append((x, 0.05 + 0.01 * k))
    S, P = 5, 2
    xs = [_t(x) for x, _ in items]
    ys = M.dsnlm_forward_batched([(x, x, h) for x, (_, h) in zip(xs, items)], S, P)
    torch.cuda.synchronize()
    for (x, h), xt, y in zip(items, xs, ys):
        y1 = M.dsnlm_forward(xt, None, S, P, h)
        assert float((y - y1).abs().max()) <= 2e-6
        yo = _oracle(x, x, S, P, h)[0]
        assert np.abs(y.cpu().numpy() - yo).max() <= TOL
    # a second call with a different batch re-uses the workspace
    ys2 = M.dsnlm_forward_batched([(xs[1], xs[1], 0.07), (xs[0], xs[0], 0.09)], S, P)
    assert float((ys2[0] - M.dsnlm_forward(xs[1], None, S, P, 0.07)).abs().max()) <= 2e-6
    assert float((ys2[1] - M.dsnlm_forward(xs[0], None, S, P, 0.09)).abs().max()) <= 2e-6
    assert M.dsnlm_forward_batched([], S, P) == []


def test_batched_full_config_properties():
    """The 64-image batch the bench times (S = 10, P = 3): every output keeps
    the image sum and stays inside [min x, max x]; two sampled images match
    the per-image launches up to summation order (2e-6)."""
    M = _gpu()
    batch = synth.config2_batch()
    xs = [_t(it.noisy) for it in batch]
    print("batched config: %d images, %d px" % (len(xs), sum(x.numel() for x in xs)), flush=True)
    ys = M.dsnlm_forward_batched([(x, x, it.h) for x, it in zip(xs, batch)], 10, 3)
    torch.cuda.synchronize()
    for x, y in zip(xs, ys):
        xd, yd = x.double(), y.double()
        assert abs(float(yd.sum() - xd.sum())) <= 2e-6 * x.numel()
        assert float(y.min()) >= float(x.min()) - 1e-6 and float(y.max()) <= float(x.max()) + 1e-6
    for k in (0, 5):
        assert float((ys[k] - M.dsnlm_forward(xs[k], None, 10, 3, batch[k].h)).abs().max()) <= 2e-6


def test_batched_bench_instance_matches_oracle():
    """The batched kernels at the configuration the bench times (S = 10,
    P = 3, h = 1.2 sigma_n, one launch per sweep over uneven images), on
    shapes of that workload the oracle can afford plus a ragged one: every
    pixel of every image, and each image's delta, m, argmax and c, against
    the FP64 oracle (Algorithm 2; steps S1-S3)."""
    M = _gpu()
    shapes = [(64, 128), (128, 128), (128, 256), (192, 384), (256, 256), (100, 150)]
    rng = np.random.default_rng(4242)
    items = []
    for k, (a, b) in enumerate(shapes):
        sig = float(rng.uniform(0.02, 0.1))
        _, x = synth.piecewise_smooth(a, b, 2100 + k, sig)
        items.append((x, 1.2 * sig))
    S, P = 10, 3
    print(f"batched S=10 P=3 vs oracle: {shapes}", flush=True)
    xs = [_t(x) for x, _ in items]
    ys = M.dsnlm_forward_batched([(x, x, h) for x, (_, h) in zip(xs, items)], S, P)
    torch.cuda.synchronize()
    for k, ((x, h), y) in enumerate(zip(items, ys)):
        yo, mo, amo, om, dl = _oracle(x, x, S, P, h)
        err = np.abs(y.cpu().numpy() - yo).max()
        assert err <= TOL, (k, err)
        m, am, c, delta = M.dsnlm_batched_state(k)
        assert abs(m - mo) <= 1e-5 * mo, (k, m, mo)
        d = np.sort(dl.ravel())
        if d[-1] - d[-2] > 1e-4 * d[-1]:
            assert am == amo, (k, am, amo)
        assert np.abs(delta.cpu().numpy() - dl).max() <= 2e-5
        assert np.abs(c.cpu().numpy() / om ** -0.5 - 1).max() <= 2e-5


def test_batched_full_config_sampled_pixels_match_oracle():
    """The 64-image batch the bench times (20.5 Mpx, images up to 1024 x 1024,
    S = 10, P = 3, h = 1.2 sigma_n, one launch per sweep), against the FP64
    oracle at full size on sampled pixels, each evaluated from its own rows of
    the matrices of steps S1-S3: at the pixel where the GPU puts the maximum
    the oracle's delta equals the GPU's m; at that pixel, two corners and two
    random pixels of every image the oracle's omega (through c), delta and
    y = W x (given m) equal the GPU's, and no sampled delta exceeds m."""
    M = _gpu()
    batch = synth.config2_batch()
    xs = [_t(it.noisy) for it in batch]
    print("batched config sampled pixels: %d images" % len(xs), flush=True)
    ys = M.dsnlm_forward_batched([(x, x, it.h) for x, it in zip(xs, batch)], 10, 3)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    for k, (it, y) in enumerate(zip(batch, ys)):
        m, am, c, delta = M.dsnlm_batched_state(k)
        n1, n2 = it.noisy.shape
        pix = [(am // n2, am % n2), (0, 0), (n1 - 1, n2 - 1),
               (int(rng.integers(n1)), int(rng.integers(n2))), (int(rng.integers(n1)), int(rng.integers(n2)))]
        q = R.dsnlm_pixels(it.noisy, it.noisy, 10, 3, it.h, pix, m)
        assert abs(q["delta"][0] - m) <= 2e-5 * m, (k, q["delta"][0], m)
        yc, cc, dc = y.cpu().numpy(), c.cpu().numpy(), delta.cpu().numpy()
        for t, (i, j) in enumerate(pix):
            assert abs(yc[i, j] - q["y"][t]) <= TOL, (k, i, j)
            assert abs(cc[i, j] * q["omega"][t] ** 0.5 - 1) <= 2e-5, (k, i, j)
            assert abs(dc[i, j] - q["delta"][t]) <= 2e-5, (k, i, j)
            assert q["delta"][t] <= m * (1 + 2e-5), (k, i, j)
