"""GPU parity of plain NLM (eq. NLM) and of Algorithm 1 with it as the
denoiser, against the FP64 oracle.  Tolerance: max-abs 2e-5 on [0, 1] images
(per step for the solver, growing linearly with the step from identical
state)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import dsnlm_ref as R
from oracle import ladmm_ref as L

pytestmark = pytest.mark.gpu

TAPS = L.gaussian_taps(9, 1.0)


def _M():
    import paper_1901_06110_amd as M
    return M


def _t(a, dtype=np.float32):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("n1,n2,S,P,h", [(64, 64, 5, 2, 0.1), (37, 131, 3, 1, 0.08), (100, 70, 10, 3, 0.05),
                                         (5, 9, 6, 2, 0.1), (1, 40, 2, 0, 0.1), (33, 65, 2, 4, 0.2),
                                         (70, 33, 0, 2, 0.1)])
def test_nlm_matches_oracle(n1, n2, S, P, h):
    M = _M()
    print(f"nlm case {n1}x{n2} S={S} P={P} h={h}", flush=True)
    _, z = synth.piecewise_smooth(n1, n2, 300 + n1 + n2, 0.05)
    _, x = synth.piecewise_smooth(n1, n2, 400 + n1 + n2, 0.05)
    y = M.dsnlm_nlm(_t(x), _t(z), S, P, h)
    ref = R.nlm_shifts(x, z, S, P, h)
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - ref).max() <= 2e-5


def test_nlm_constant_and_identity_on_gpu():
    M = _M()
    rng = np.random.default_rng(3)
    z = rng.random((45, 77)).astype(np.float32)
    y = M.dsnlm_nlm(_t(np.full((45, 77), 0.37)), _t(z), 4, 2, 0.1)
    torch.cuda.synchronize()
    assert np.abs(y.cpu().numpy() - np.float32(0.37)).max() <= 1e-6
    x = rng.random((45, 77)).astype(np.float32)
    y = M.dsnlm_nlm(_t(x), _t(z), 4, 2, 1e-4)  # every off-diagonal kernel underflows
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), x)


def test_sr_steps_with_plain_nlm_match_oracle():
    M = _M()
    n, S, P, steps = 48, 5, 2, 4
    clean, _ = synth.piecewise_smooth(n, n, 31, 0.0)
    rng = np.random.default_rng(32)
    y = (L.sr_forward(clean, TAPS, 2) + 0.01 * rng.standard_normal((n // 2, n // 2))).astype(np.float32)
    x0 = synth.bicubic_upsample(y, 2)
    gamma = np.float32(1.0 / 0.3321609)
    lam, rho = np.float32(1e-2), np.float32(1.0)
    h = float(np.float32(math.sqrt(lam / rho)))
    taps32 = TAPS.astype(np.float32)
    grad_f = lambda v: L.sr_adjoint(L.sr_forward(v, taps32, 2) - y, taps32, 2, v.shape)
    rec = []
    L.ladmm(x0, grad_f, alpha=1.0 / float(gamma), rho=float(rho), S=S, P=P, h=h, iters=steps,
            freeze_after=steps, v0=x0, u0=np.zeros_like(x0), record=rec,
            denoise=lambda zz, gg: R.nlm_shifts(zz, zz, S, P, h))
    taps = np.ascontiguousarray(TAPS, dtype=np.float32)
    op = M.SROperator(n1=n, n2=n, taps=taps, factor=2, y=_t(y), boundary=0)
    prm = M.LadmmParams(lam=float(lam), rho=float(rho), gamma=float(gamma), S=S, P=P, freeze_after=1,
                        iters=steps, denoiser=1)
    x, v, u = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    w = None
    for k in range(1, steps + 1):
        w = M.ladmm_step(op, prm, k, w, x, v, u)
        torch.cuda.synchronize()
        xo, vo, uo, _ = rec[k - 1]
        tol = 2e-5 * k
        assert np.abs(x.cpu().numpy() - xo).max() <= tol, k
        assert np.abs(v.cpu().numpy() - vo).max() <= tol, k
        assert np.abs(u.cpu().numpy() - uo).max() <= tol, k
    # the solver gives the same iterates (no frozen phase, no graph)
    x2, v2, u2 = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    M.ladmm_solve(op, prm, x2, v2, u2)
    torch.cuda.synchronize()
    assert torch.equal(x2, x) and torch.equal(v2, v) and torch.equal(u2, u)
