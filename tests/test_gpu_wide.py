"""GPU parity of the wide-patch passes (5 < P <= 15, patch sides 13..31, the
patch sizes of Table 1) against the FP64 oracle, through the C ABI.

Tolerance: max-abs 2e-5 on [0, 1] images, as for the other forward paths.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dsnlm_ref as R

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _M():
    import paper_1901_06110_amd as M
    return M


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# several 32 x 32 tiles with ragged tails, S >= size, P up to the maximum
CASES = [(40, 70, 4, 6, 0.15), (45, 33, 3, 8, 0.2), (50, 70, 6, 11, 0.2), (20, 24, 7, 15, 0.3),
         (33, 17, 2, 14, 0.25)]


@pytest.mark.parametrize("n1,n2,S,P,h", CASES)
def test_wide_forward_matches_oracle(n1, n2, S, P, h):
    M = _M()
    print(f"wide case {n1}x{n2} S={S} P={P}", flush=True)
    _, z = synth.piecewise_smooth(n1, n2, 800 + n1, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, 900 + n2, 0.05)
    y, w = M.dsnlm_forward(_t(x), _t(z), S, P, h, keep=True)
    ref = R.dsnlm_shifts(x, z, S, P, h)
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - ref["y"].numpy()).max() <= TOL
    assert np.abs(w.array(1).cpu().numpy() - ref["delta"].numpy()).max() <= TOL
    m, am = w.scalars()
    assert abs(m - float(ref["m"])) <= TOL * float(ref["m"])


def test_wide_build_apply_equals_forward_and_brute():
    """Three sweeps (build, then apply) give exactly the fused forward; the
    brute-force comparator agrees within the tolerance."""
    M = _M()
    S, P, h = 5, 9, 0.2
    _, z = synth.piecewise_smooth(48, 66, 31, 0.05)
    _, x = synth.piecewise_smooth(48, 66, 32, 0.05)
    w = M.dsnlm_build_weights(_t(z), S, P, h)
    y1 = M.dsnlm_apply(w, _t(x))
    y2 = M.dsnlm_forward(_t(x), _t(z), S, P, h)
    yb = M.dsnlm_forward_brute(_t(x), _t(z), S, P, h)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    assert float((yb - y2).abs().max()) <= TOL


def test_wide_properties_at_the_largest_sizes():
    """S = 24, P = 15 on a 128 x 96 image: constants are fixed points, the mean
    is preserved (W is doubly stochastic) and y stays within [min x, max x],
    up to FP32 rounding over windows of 49 x 49 terms (5e-6)."""
    M = _M()
    S, P, h = 24, 15, 0.2
    _, z = synth.piecewise_smooth(128, 96, 41, 0.05)
    _, x = synth.piecewise_smooth(128, 96, 42, 0.05)
    c = torch.full((128, 96), 0.37, device="cuda")
    yc = M.dsnlm_forward(c, _t(z), S, P, h)
    y = M.dsnlm_forward(_t(x), _t(z), S, P, h).double()
    torch.cuda.synchronize()
    assert float((yc - 0.37).abs().max()) <= 5e-6
    xd = _t(x).double()
    assert abs(float(y.mean() - xd.mean())) <= 5e-6
    assert float(y.min()) >= float(xd.min()) - 5e-6 and float(y.max()) <= float(xd.max()) + 5e-6


def test_wide_patches_rejected_where_unsupported():
    """The backward, the batched form and LADMM keep P <= 5."""
    M = _M()
    _, x = synth.piecewise_smooth(40, 40, 51, 0.05)
    y, w = M.dsnlm_forward(_t(x), None, 3, 6, 0.2, keep=True)
    with pytest.raises(M.api._lib.DsnlmError):
        M.dsnlm_apply_backward(w, _t(x), torch.ones_like(y))
    with pytest.raises(M.api._lib.DsnlmError):
        M.dsnlm_forward_batched([(_t(x), _t(x), 0.2)], 3, 6)
