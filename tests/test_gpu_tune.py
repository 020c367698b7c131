"""The autotuner and the shift-group split of single-image sweeps.

A single-image half-window sweep splits each tile's shifts into equal
contiguous ranges (one block each).  Every group count from 1 to 8, including
counts that end a range in the middle of a dx column, must give the FP64
oracle's result (eqs. NLM, S1-S3) for the forward, a frozen apply and the
input gradient (sweep C).  dsnlm_tune then picks schedules and a group count
by timing; the tuned configuration must give the oracle's result as well.
Both tests restore the tables they change.
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
def tables():
    import paper_1901_06110_amd as M
    from paper_1901_06110_amd import _lib
    lib = _lib.get()
    saved_v, saved_g = {}, {}

    def remember(n1, n2, S, P):
        for kind in range(4):
            cur = C.c_int()
            _lib.check(lib.dsnlm_tune_get(kind, S, P, C.byref(cur)))
            saved_v.setdefault((kind, S, P), cur.value)
        saved_g.setdefault((n1, n2, S, P), 0)  # the tests start from the rule

    yield M, lib, remember
    for (kind, S, P), v in saved_v.items():
        lib.dsnlm_tune_set(kind, S, P, v)
    for (n1, n2, S, P), g in saved_g.items():
        lib.dsnlm_tune_set_groups(n1, n2, S, P, g)


def _check_forward_apply_grad(M, x_np, S, P, h):
    ref = R.dsnlm_shifts(x_np, x_np, S, P, h)
    x = _t(x_np)
    y, w = M.dsnlm_forward(x, None, S, P, h, keep=True)
    err_f = float(np.abs(y.cpu().numpy() - ref["y"].detach().numpy()).max())
    # frozen apply of the same weights to another image
    x2_np = np.ascontiguousarray(x_np[::-1, :])
    y2 = M.dsnlm_apply(w, _t(x2_np))
    ref2 = R.dsnlm_shifts(x2_np, x_np, S, P, h)["y"].detach().numpy()
    err_a = float(np.abs(y2.cpu().numpy() - ref2).max())
    # input gradient W ybar (sweep C) against the dense W of the oracle (relative error)
    yb = np.random.default_rng(5).standard_normal(x_np.shape).astype(np.float32)
    M.dsnlm_forward(x, _t(x_np), S, P, h, weights=w)
    dx, _, _ = M.dsnlm_apply_backward(w, x, _t(yb), need_dguide=False, need_dh=False)
    Wd = R.dense_weights(x_np.astype(np.float64), S, P, h)["W"]
    gref = (Wd.T @ yb.astype(np.float64).ravel()).reshape(x_np.shape)
    err_g = float(np.abs(dx.cpu().numpy() - gref).max()) / float(np.abs(gref).max())
    return err_f, err_a, err_g


@pytest.mark.parametrize("groups", [1, 2, 3, 5, 7, 8])
def test_every_group_count_matches_oracle(tables, groups):
    M, lib, remember = tables
    n1, n2, S, P, h = 40, 70, 5, 2, 0.1
    remember(n1, n2, S, P)
    from paper_1901_06110_amd import _lib
    _lib.check(lib.dsnlm_tune_set_groups(n1, n2, S, P, groups))
    got = C.c_int()
    _lib.check(lib.dsnlm_tune_get_groups(n1, n2, S, P, C.byref(got)))
    assert got.value == groups
    _, x_np = synth.piecewise_smooth(n1, n2, seed=8100 + groups, sigma_n=0.05)
    print(f"groups {groups}: {n1}x{n2} S={S} P={P}", flush=True)
    err_f, err_a, err_g = _check_forward_apply_grad(M, x_np, S, P, h)
    torch.cuda.synchronize()
    assert err_f <= TOL and err_a <= TOL, (err_f, err_a)
    assert err_g <= 1e-4, err_g


def test_tuned_configuration_matches_oracle(tables):
    M, lib, remember = tables
    from paper_1901_06110_amd import _lib
    n1, n2, S, P, h = 96, 150, 10, 3, 0.08
    remember(n1, n2, S, P)
    _, x_np = synth.piecewise_smooth(n1, n2, seed=8200, sigma_n=0.05)
    x = _t(x_np)
    print(f"tune {n1}x{n2} S={S} P={P}", flush=True)
    _lib.check(lib.dsnlm_tune(C.c_void_p(x.data_ptr()), n1, n2, S, P, h, 3,
                              C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    chosen = []
    for kind in range(4):
        v = C.c_int()
        _lib.check(lib.dsnlm_tune_get(kind, S, P, C.byref(v)))
        assert 0 <= v.value <= 3
        chosen.append(v.value)
    g = C.c_int()
    _lib.check(lib.dsnlm_tune_get_groups(n1, n2, S, P, C.byref(g)))
    assert 1 <= g.value <= 8
    print(f"tuned variants {chosen}, groups {g.value}", flush=True)
    err_f, err_a, err_g = _check_forward_apply_grad(M, x_np, S, P, h)
    torch.cuda.synchronize()
    assert err_f <= TOL and err_a <= TOL, (err_f, err_a)
    assert err_g <= 1e-4, err_g
