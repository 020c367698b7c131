"""GPU parity of the hand-written backward of y = W(guide, h) x.

References: torch CPU float64 autograd through the oracle's shift loop, and
central finite differences of the FP64 oracle (step 1e-3) on 32x32 crops.
Bar: relative error <= 1e-3 (max |gpu - ref| / max |ref|).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dsnlm_ref as R
from oracle import grad_ref as G

pytestmark = pytest.mark.gpu


def _M():
    import paper_1901_06110_amd as M
    return M


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-30))


def _case(n1, n2, seed, sep_guide=True):
    clean, x = synth.piecewise_smooth(n1, n2, seed, 0.05)
    z = synth.piecewise_smooth(n1, n2, seed + 50, 0.05)[1] if sep_guide else x
    return clean, x, z


CASES = [(32, 32, 7, 3, 0.1), (29, 41, 3, 1, 0.08), (40, 24, 5, 2, 0.12), (33, 70, 10, 3, 0.1),
         (12, 12, 6, 2, 0.15), (40, 70, 16, 2, 0.1), (28, 30, 18, 2, 0.12), (26, 30, 13, 4, 0.12),
         (24, 26, 14, 5, 0.15), (20, 37, 3, 0, 0.1), (1, 40, 2, 0, 0.1), (3, 45, 4, 1, 0.1)]


@pytest.mark.parametrize("n1,n2,S,P,h", CASES)
def test_backward_matches_fp64_autograd(n1, n2, S, P, h):
    M = _M()
    print(f"backward case {n1}x{n2} S={S} P={P} h={h}", flush=True)
    clean, x, z = _case(n1, n2, 300 + n1 + n2)
    y, w = M.dsnlm_forward(_t(x), _t(z), S, P, h, keep=True)
    ybar = 2.0 * (y.cpu().numpy().astype(np.float64) - clean)  # loss ||W x - clean||^2
    ref = G.autograd_grads(x, z, S, P, h, ybar)
    d = np.sort(ref["delta"].ravel())
    assert d[-1] - d[-2] >= 1e-4 * d[-1], "tie in the maximum row sum"
    dx, dg, dh = M.dsnlm_apply_backward(w, _t(x), _t(ybar))
    torch.cuda.synchronize()
    assert _rel(dx.cpu().numpy(), ref["dx"]) <= 1e-4
    assert _rel(dg.cpu().numpy(), ref["dz"]) <= 1e-3
    assert abs(float(dh.cpu()) - ref["dh"]) <= 1e-3 * abs(ref["dh"])


def test_backward_central_fd_32x32_crop():
    """Config of the differentiated denoiser (S = 7, P = 3, h = 0.1) on a 32x32
    crop: loss ||W(g, h) x - x_clean||^2, FD of the FP64 oracle, step 1e-3."""
    M = _M()
    batch = synth.config3_batch(count=1, n=256)
    clean, noisy = batch[0]
    clean, x = clean[100:132, 60:92], noisy[100:132, 60:92]
    z = x.copy()
    S, P, h = 7, 3, 0.1
    xt = _t(x).requires_grad_(True)
    zt = _t(z).requires_grad_(True)
    ht = torch.tensor(h, device="cuda", requires_grad=True)
    y = M.dsnlm(xt, zt, ht, S, P)
    loss = ((y.double() - _t(clean).double()) ** 2).sum()
    loss.backward()
    rng = np.random.default_rng(0)
    idx = rng.choice(x.size, 12, replace=False)
    f = lambda zz: G.loss_value(x, zz, S, P, h, target=clean)
    fd = G.central_fd(f, z, idx, step=1e-3)
    an = zt.grad.cpu().numpy().ravel()[idx]
    scale = max(np.abs(zt.grad.cpu().numpy()).max(), 1e-12)
    assert np.abs(fd - an).max() <= 1e-3 * scale
    fdx = G.central_fd(lambda xx: G.loss_value(xx, z, S, P, h, target=clean), x, idx, step=1e-3)
    sx = max(np.abs(xt.grad.cpu().numpy()).max(), 1e-12)
    assert np.abs(fdx - xt.grad.cpu().numpy().ravel()[idx]).max() <= 1e-3 * sx
    fdh = G.central_fd(lambda hh: G.loss_value(x, z, S, P, hh, target=clean), h, None, step=1e-4)[0]
    assert abs(float(ht.grad) - fdh) <= 1e-3 * abs(fdh)


def test_self_guided_gradient_sums_both_paths():
    """guide = x: the gradient is the input path plus the guide path."""
    M = _M()
    clean, x, _ = _case(24, 30, 77, sep_guide=False)
    S, P, h = 4, 2, 0.1
    xt = _t(x).requires_grad_(True)
    y = M.dsnlm(xt, None, 0.1, S, P)
    ((y.double() - _t(clean).double()) ** 2).sum().backward()
    ybar = 2.0 * (y.detach().cpu().numpy().astype(np.float64) - clean)
    ref = G.autograd_grads(x, x, S, P, h, ybar)
    assert _rel(xt.grad.cpu().numpy(), ref["dx"] + ref["dz"]) <= 1e-3


def test_backward_c3_batch_shape_runs_and_is_deterministic():
    """Eight 256x256 images at S = 7, P = 3: gradients finite, two backward
    runs bit-identical (fixed-order reductions, no atomics)."""
    M = _M()
    batch = synth.config3_batch()
    for clean, noisy in batch[:2]:
        y, w = M.dsnlm_forward(_t(noisy), _t(noisy), 7, 3, 0.1, keep=True)
        yb = 2 * (y - _t(clean))
        a = M.dsnlm_apply_backward(w, _t(noisy), yb)
        b = M.dsnlm_apply_backward(w, _t(noisy), yb)
        torch.cuda.synchronize()
        for u, v in zip(a, b):
            assert torch.isfinite(u).all()
            assert torch.equal(u, v)


@pytest.mark.parametrize("S,P", [(7, 3), (4, 1), (10, 2), (10, 3), (16, 3)])
def test_batched_backward_matches_fp64_autograd(S, P):
    """One batched forward and backward over images of uneven sizes (several
    tiles and ragged tails): every image's gradients against the FP64
    autograd reference, and against the single-image backward.  S = 10,
    P = 3 is the instance the bench's forward+backward times."""
    M = _M()
    shapes = [(32, 32, 0.1), (29, 71, 0.08), (70, 45, 0.12), (12, 12, 0.15)]
    imgs, refs = [], []
    for k, (n1, n2, h) in enumerate(shapes):
        clean, x, z = _case(n1, n2, 900 + 7 * k)
        imgs.append((clean, x, z, h))
    print(f"batched backward S={S} P={P} shapes={shapes}", flush=True)
    # the forward's inputs must stay alive and unchanged until the backward
    dev = [(_t(z), _t(x), h) for _, x, z, h in imgs]
    ys = M.dsnlm_forward_batched(dev, S, P)
    ybars = []
    for (clean, x, z, h), y in zip(imgs, ys):
        ybar = 2.0 * (y.cpu().numpy().astype(np.float64) - clean)
        ybars.append(ybar)
        ref = G.autograd_grads(x, z, S, P, h, ybar)
        d = np.sort(ref["delta"].ravel())
        assert d[-1] - d[-2] >= 1e-4 * d[-1], "tie in the maximum row sum"
        refs.append(ref)
    out = M.dsnlm_backward_batched([_t(yb) for yb in ybars])
    torch.cuda.synchronize()
    for (clean, x, z, h), ybar, ref, (dx, dg, dh) in zip(imgs, ybars, refs, out):
        assert _rel(dx.cpu().numpy(), ref["dx"]) <= 1e-4
        assert _rel(dg.cpu().numpy(), ref["dz"]) <= 1e-3
        assert abs(float(dh.cpu()) - ref["dh"]) <= 1e-3 * abs(ref["dh"])
        _, w = M.dsnlm_forward(_t(x), _t(z), S, P, h, keep=True)
        dx1, dg1, dh1 = M.dsnlm_apply_backward(w, _t(x), _t(ybar))
        torch.cuda.synchronize()
        assert _rel(dx.cpu().numpy(), dx1.cpu().numpy()) <= 1e-5
        assert _rel(dg.cpu().numpy(), dg1.cpu().numpy()) <= 1e-4


def test_batched_backward_input_gradient_only_and_errors():
    M = _M()
    S, P = 5, 2
    data = [_case(40, 37, 950), _case(17, 66, 951)]
    dev = [(_t(z), _t(x), 0.1) for _, x, z in data]
    ys = M.dsnlm_forward_batched(dev, S, P)
    ybars = [np.random.default_rng(k).standard_normal(y.shape) for k, y in enumerate(ys)]
    out = M.dsnlm_backward_batched([_t(yb) for yb in ybars], need_dguide=False, need_dh=False)
    torch.cuda.synchronize()
    for (_, x, z), yb, (dx, dg, dh) in zip(data, ybars, out):
        assert dg is None and dh is None
        Wd = R.dense_weights(z, S, P, 0.1)["W"]
        ref = (Wd @ yb.ravel()).reshape(yb.shape)
        assert _rel(dx.cpu().numpy(), ref) <= 1e-4
    with pytest.raises(M.api._lib.DsnlmError):
        M.dsnlm_backward_batched([_t(ybars[0])])


def test_batched_backward_full_size_directional_derivatives():
    """The differentiated denoiser's full batch (8 x 256^2, S = 7, P = 3), at a
    size the FP64 autograd reference cannot reach: for the loss L = <ybar, y>
    (linear in y), the batched backward's gradients must match central
    differences of the GPU forward itself along chosen directions:
      guide: a +-1 pattern on a 24 x 24 window far from the argmax pixel s*
             (m and s* do not move, so only pixels near the window change);
      x:     <dx, u> = <ybar, W u> for a random u (W is symmetric);
      h:     a step of 1e-3 in h.
    The sums are taken in FP64 on the host."""
    M = _M()
    S, P, h = 7, 3, 0.1
    batch = synth.config3_batch()
    dev = [(_t(noisy), _t(noisy), h) for _, noisy in batch]
    ys = M.dsnlm_forward_batched(dev, S, P)
    rng = np.random.default_rng(2024)
    ybars = [_t(rng.standard_normal(y.shape)) for y in ys]
    out = M.dsnlm_backward_batched(ybars)
    torch.cuda.synchronize()

    def loss(z, x, hh, yb):
        y = M.dsnlm_forward(x, z, S, P, hh)
        return float((y.double() * yb.double()).sum())

    for k in (0, 5):
        z, x, _ = dev[k]
        yb = ybars[k]
        dx, dg, dh = out[k]
        _, w = M.dsnlm_forward(x, z, S, P, h, keep=True)
        m, am = w.scalars()
        si, sj = divmod(am, z.shape[1])
        print(f"full-size directional check image {k}: s* = ({si}, {sj})", flush=True)
        i0 = 16 if si >= 128 else 216
        j0 = 16 if sj >= 128 else 216
        v = torch.zeros_like(z)
        v[i0:i0 + 24, j0:j0 + 24] = _t(rng.choice([-1.0, 1.0], size=(24, 24)))
        eps = 4e-3
        for sgn in (1.0, -1.0):
            _, wp = M.dsnlm_forward(x, z + sgn * eps * v, S, P, h, keep=True)
            assert wp.scalars()[1] == am
        fd = (loss(z + eps * v, x, h, yb) - loss(z - eps * v, x, h, yb)) / (2 * eps)
        an = float((dg.double() * v.double()).sum())
        assert abs(fd - an) <= 2e-3 * abs(an), (fd, an)
        u = _t(rng.standard_normal(z.shape))
        wu = M.dsnlm_forward(u, z, S, P, h)
        lhs = float((dx.double() * u.double()).sum())
        rhs = float((yb.double() * wu.double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * float(dx.double().abs().sum()), (lhs, rhs)
        dhf = (loss(z, x, h + 1e-3, yb) - loss(z, x, h - 1e-3, yb)) / 2e-3
        print(f"  guide {an:.6g} vs fd {fd:.6g}; x {lhs:.8g} vs {rhs:.8g}; h {float(dh.cpu()):.6g} vs fd {dhf:.6g}",
              flush=True)
        assert abs(float(dh.cpu()) - dhf) <= 2e-3 * abs(dhf), (float(dh.cpu()), dhf)


def test_batched_backward_full_config_sampled_pixels():
    """The backward the bench times: the 64-image batch (20.5 Mpx, S = 10,
    P = 3, h = 1.2 sigma_n) with every gradient requested.  W is symmetric,
    so x-bar = W y-bar; at two corners and three random pixels of every image
    it must equal the FP64 oracle's rows of steps S1-S3 applied to y-bar
    (given the image's m), and over each whole image sum(x-bar) = sum(y-bar)
    (the columns of W sum to one); h-bar is finite."""
    M = _M()
    batch = synth.config2_batch()
    xs = [_t(it.noisy) for it in batch]
    print("batched backward full config: %d images" % len(xs), flush=True)
    M.dsnlm_forward_batched([(x, x, it.h) for x, it in zip(xs, batch)], 10, 3)
    rng = np.random.default_rng(91)
    ybars = [rng.standard_normal(it.noisy.shape).astype(np.float32) for it in batch]
    out = M.dsnlm_backward_batched([_t(yb) for yb in ybars])
    torch.cuda.synchronize()
    for k, (it, yb, (dx, dg, dh)) in enumerate(zip(batch, ybars, out)):
        m, _, _, _ = M.dsnlm_batched_state(k)
        n1, n2 = it.noisy.shape
        dxc = dx.cpu().numpy()
        assert abs(float(dxc.astype(np.float64).sum()) - float(yb.astype(np.float64).sum())) <= 1e-5 * yb.size, k
        assert np.isfinite(float(dh.cpu())) and bool(torch.isfinite(dg).all()), k
        pix = [(0, 0), (n1 - 1, n2 - 1)] + [(int(rng.integers(n1)), int(rng.integers(n2))) for _ in range(3)]
        q = R.dsnlm_pixels(yb, it.noisy, 10, 3, it.h, pix, m)
        scale = float(np.abs(yb).max())
        for t, (i, j) in enumerate(pix):
            assert abs(dxc[i, j] - q["y"][t]) <= 1e-4 * scale, (k, i, j, dxc[i, j], q["y"][t])
