"""Every sweep schedule gives the oracle's result.

The sweeps have four compiled schedules selectable per sweep kind (0 plain,
1 software-pipelined, 2 grouped register window, 3 half window with a gather);
3 is the default.  Each is pinned in turn for every kind and checked against
the FP64 oracle (forward, build + frozen apply) and against W ybar from the
oracle's dense W (input gradient, which runs sweep C).
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from oracle import dsnlm_ref as R

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture
def pin():
    import paper_1901_06110_amd as M
    from paper_1901_06110_amd import _lib
    lib = _lib.get()
    saved = {}

    def set_all(S, P, v):
        for kind in range(4):
            cur = C.c_int()
            _lib.check(lib.dsnlm_tune_get(kind, S, P, C.byref(cur)))
            saved.setdefault((kind, S, P), cur.value)
            _lib.check(lib.dsnlm_tune_set(kind, S, P, v))
    yield M, set_all
    for (kind, S, P), v in saved.items():
        lib.dsnlm_tune_set(kind, S, P, v)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("n1,n2,S,P,h", [(70, 131, 10, 3, 0.05), (33, 40, 4, 2, 0.1)])
def test_every_schedule_matches_oracle(pin, variant, n1, n2, S, P, h):
    M, set_all = pin
    set_all(S, P, variant)
    print(f"variant {variant} case {n1}x{n2} S={S} P={P}", flush=True)
    _, z = synth.piecewise_smooth(n1, n2, 700 + n1, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, 800 + n2, 0.05)
    y, w = M.dsnlm_forward(_t(x), _t(z), S, P, h, keep=True)
    yo = R.dsnlm_shifts(x, z, S, P, h)["y"].numpy()
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - yo).max() <= TOL
    # frozen apply of the built weights to another image
    _, x2 = synth.piecewise_smooth(n1, n2, 900 + n2, 0.05)
    wb = M.dsnlm_build_weights(_t(z), S, P, h)
    y2 = M.dsnlm_apply(wb, _t(x2))
    y2o = R.dsnlm_shifts(x2, z, S, P, h)["y"].numpy()
    torch.cuda.synchronize()
    assert np.abs(y2.cpu().numpy() - y2o).max() <= TOL
    if n1 * n2 <= 1500:
        ybar = np.random.default_rng(variant).standard_normal((n1, n2))
        dx, _, _ = M.dsnlm_apply_backward(w, _t(x), _t(ybar), need_dguide=False, need_dh=False)
        Wd = R.dense_weights(z, S, P, h)["W"]
        ref = (Wd @ ybar.ravel()).reshape(n1, n2)
        torch.cuda.synchronize()
        assert np.abs(dx.cpu().numpy() - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("pass_b_variant", [0, 2])
def test_half_apply_after_full_window_build(pin, pass_b_variant):
    """The half-window apply keeps one channel (the sum of a c x) and takes
    the sum of a c, fixed with the weights, from the build: pass B's own sum
    when pass B ran on the half window, else delta / c.  With pass B pinned to
    a full-window schedule and the apply left on the half window, the apply
    must still give the oracle's result."""
    from paper_1901_06110_amd import _lib
    M, _ = pin
    lib = _lib.get()
    n1, n2, S, P, h = 70, 131, 10, 3, 0.05
    set_all = pin[1]
    set_all(S, P, 3)  # records and restores every kind's entry
    _lib.check(lib.dsnlm_tune_set(1, S, P, pass_b_variant))
    print(f"pass B variant {pass_b_variant}, half apply, {n1}x{n2} S={S} P={P}", flush=True)
    _, z = synth.piecewise_smooth(n1, n2, 710, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, 810, 0.05)
    wb = M.dsnlm_build_weights(_t(z), S, P, h)
    y = M.dsnlm_apply(wb, _t(x))
    yo = R.dsnlm_shifts(x, z, S, P, h)["y"].numpy()
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - yo).max() <= TOL
