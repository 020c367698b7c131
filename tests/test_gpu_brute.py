"""The brute-force comparator (patch distances summed directly) gives the
oracle's DSG-NLM output, like the fast path.  Tolerance: max-abs 2e-5."""
import numpy as np
import pytest
import torch

import synth
from oracle import dsnlm_ref as R

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n1,n2,S,P,h", [(64, 64, 5, 2, 0.1), (37, 71, 10, 3, 0.05), (5, 9, 6, 2, 0.1),
                                         (40, 33, 3, 5, 0.2)])
def test_brute_matches_oracle_and_fast_path(n1, n2, S, P, h):
    import paper_1901_06110_amd as M
    print(f"brute case {n1}x{n2} S={S} P={P}", flush=True)
    _, z = synth.piecewise_smooth(n1, n2, 500 + n1, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, 600 + n2, 0.05)
    yb = M.dsnlm_forward_brute(_t(x), _t(z), S, P, h)
    yf = M.dsnlm_forward(_t(x), _t(z), S, P, h)
    yo = R.dsnlm_shifts(x, z, S, P, h)["y"].numpy()
    torch.cuda.synchronize()
    assert np.abs(yb.cpu().numpy() - yo).max() <= 2e-5
    assert np.abs(yb.cpu().numpy() - yf.cpu().numpy()).max() <= 2e-5
