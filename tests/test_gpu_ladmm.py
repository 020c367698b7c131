"""GPU parity of linearized PnP-ADMM (Algorithm 1) against the FP64 oracle."""
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


def _sr_op(M, n1, n2, y=None, boundary=0, factor=2, taps=TAPS):
    return M.SROperator(n1=n1, n2=n2, taps=np.asarray(taps, np.float32), factor=factor,
                        y=y, boundary=boundary)


BNAME = {0: "symmetric", 1: "periodic"}


@pytest.mark.parametrize("boundary", [0, 1])
@pytest.mark.parametrize("shape,factor", [((40, 36), 2), ((33, 29), 2), ((64, 64), 2), ((30, 45), 3)])
def test_sr_operator_and_gradient(boundary, shape, factor):
    M = _M()
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, shape).astype(np.float32)
    op = _sr_op(M, *shape, boundary=boundary, factor=factor)
    ax = M.ladmm_apply_forward(op, _t(x)).cpu().numpy()
    ref = L.sr_forward(x, TAPS.astype(np.float32), factor, BNAME[boundary])
    assert ax.shape == ref.shape
    assert np.abs(ax - ref).max() <= 1e-6
    y = rng.uniform(0, 1, ref.shape).astype(np.float32)
    op.y = _t(y)
    g = M.ladmm_gradient(op, _t(x)).cpu().numpy()
    gref = L.sr_adjoint(ref - y, TAPS.astype(np.float32), factor, shape, BNAME[boundary])
    assert np.abs(g - gref).max() <= 2e-6


def test_operator_norm():
    M = _M()
    beta = float((TAPS * (-1.0) ** np.arange(9)).sum())
    op = _sr_op(M, 32, 32, boundary=1)
    assert abs(M.ladmm_operator_norm2(op, 1500) - 0.25 * (1 + beta * beta) ** 2) <= 2e-5
    A = L.sr_dense((32, 32), TAPS, 2, "symmetric")
    op = _sr_op(M, 32, 32, boundary=0)
    assert abs(M.ladmm_operator_norm2(op, 1500) - np.linalg.norm(A, 2) ** 2) <= 2e-5


def test_spi_gradient():
    M = _M()
    K, eta = 16, 4.0
    clean, uni = synth.config4_batch(count=1, n=48, K=K)[0]
    ones = L.spi_counts(clean, uni, eta)
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(0, 1, (40, 48)), np.full((8, 48), 1e-7)]).astype(np.float32)
    op = M.SPIOperator(n1=48, n2=48, ones=_t(ones, np.uint8), K=K, eta=eta)
    g = M.ladmm_gradient(op, _t(x)).cpu().numpy()
    gref = L.spi_grad(x, ones, K, eta)
    assert np.all(np.abs(g - gref) <= 1e-5 * np.maximum(1.0, np.abs(gref)))


def _oracle_steps(x0, v0, u0, grad_f, alpha, rho, S, P, h, k0, nsteps, lo=0.0, hi=1.0):
    rec = []
    out = L.ladmm(x0, grad_f, alpha=alpha, rho=rho, S=S, P=P, h=h, iters=nsteps,
                  freeze_after=k0, lo=lo, hi=hi, v0=v0, u0=u0, record=rec)
    return out, rec


def _sr_problem(n, seed, S, P):
    clean, _ = synth.piecewise_smooth(n, n, seed, 0.0)
    rng = np.random.default_rng(seed + 1)
    y = (L.sr_forward(clean, TAPS, 2) + 0.01 * rng.standard_normal((n // 2, n // 2))).astype(np.float32)
    x0 = synth.bicubic_upsample(y, 2)
    return clean, y, x0


@pytest.mark.parametrize("n,S,P,k0,steps", [(40, 3, 1, 1, 3), (64, 10, 3, 5, 6)])
def test_sr_steps_match_oracle(n, S, P, k0, steps):
    """Iterations from the same state: adaptive (k <= k0) then frozen weights."""
    M = _M()
    clean, y, x0 = _sr_problem(n, 21, S, P)
    gamma = np.float32(1.0 / 0.3321609)
    lam, rho = np.float32(1e-2), np.float32(1.0)
    h = float(np.float32(math.sqrt(lam / rho)))
    taps32 = TAPS.astype(np.float32)
    grad_f = lambda v: L.sr_adjoint(L.sr_forward(v, taps32, 2) - y, taps32, 2, v.shape)
    out, rec = _oracle_steps(x0, x0, np.zeros_like(x0), grad_f, 1.0 / float(gamma), float(rho),
                             S, P, h, k0, steps)
    op = _sr_op(M, n, n, y=_t(y))
    prm = M.LadmmParams(lam=float(lam), rho=float(rho), gamma=float(gamma), S=S, P=P,
                        freeze_after=k0, iters=steps)
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


def test_spi_steps_match_oracle():
    M = _M()
    K, eta, S, P, n = 16, 4.0, 7, 2, 48
    clean, uni = synth.config4_batch(count=1, n=n, K=K)[0]
    ones = L.spi_counts(clean, uni, eta)
    x0 = np.clip(L.spi_ml(ones, K, eta), 0, 1).astype(np.float32)
    lam, rho, gamma = 1e-2, 1.0, 1.0 / 16.0
    h = float(np.float32(math.sqrt(lam / rho)))
    grad_f = lambda v: L.spi_grad(v, ones, K, eta)
    out, rec = _oracle_steps(x0, x0, np.zeros_like(x0), grad_f, 16.0, rho, S, P, h, 2, 3)
    op = M.SPIOperator(n1=n, n2=n, ones=_t(ones, np.uint8), K=K, eta=eta)
    prm = M.LadmmParams(lam=lam, rho=rho, gamma=gamma, S=S, P=P, freeze_after=2, iters=3)
    x, v, u = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    w = None
    for k in range(1, 4):
        w = M.ladmm_step(op, prm, k, w, x, v, u)
        torch.cuda.synchronize()
        xo, vo, uo, _ = rec[k - 1]
        assert np.abs(x.cpu().numpy() - xo).max() <= 2e-5 * k
        assert np.abs(v.cpu().numpy() - vo).max() <= 2e-5 * k
        assert np.abs(u.cpu().numpy() - uo).max() <= 2e-5 * k


def test_solve_equals_steps_and_checkpoints():
    """ladmm_solve (frozen iterations replayed from a graph) gives bit-equal
    states, residuals and checkpoints to the same iterations one by one."""
    M = _M()
    n, S, P, k0, iters = 48, 5, 2, 3, 9
    clean, y, x0 = _sr_problem(n, 31, S, P)
    op = _sr_op(M, n, n, y=_t(y))
    prm = M.LadmmParams(lam=1e-2, rho=1.0, gamma=1.0 / 0.3321609, S=S, P=P, h=0.05,
                        freeze_after=k0, iters=iters)
    x1, v1, u1 = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    res = torch.zeros((iters, 2), device="cuda")
    ck = torch.zeros((iters, 4, n, n), device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        M.ladmm_solve(op, prm, x1, v1, u1, residuals=res, checkpoints=ck)
    torch.cuda.synchronize()
    x2, v2, u2 = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    w = None
    for k in range(1, iters + 1):
        u_prev = u2.clone()
        w = M.ladmm_step(op, prm, k, w, x2, v2, u2)
        torch.cuda.synchronize()
        assert torch.equal(ck[k - 1, 0], x2) and torch.equal(ck[k - 1, 1], v2)
        assert torch.equal(ck[k - 1, 2], u2)
        assert torch.equal(ck[k - 1, 3], x2 + u_prev)  # the denoiser input
    assert torch.equal(x1, x2) and torch.equal(v1, v2) and torch.equal(u1, u2)
    # residuals: RMS of x - v and of rho (v_k - v_{k-1})
    r = res.cpu().numpy()
    assert np.all(np.isfinite(r))
    xv = (ck[-1, 0] - ck[-1, 1]).double()
    assert abs(r[-1, 0] - float(xv.pow(2).mean().sqrt())) <= 1e-6 + 1e-4 * r[-1, 0]
    dv = (ck[-1, 1] - ck[-2, 1]).double()
    assert abs(r[-1, 1] - float(dv.pow(2).mean().sqrt())) <= 1e-6 + 1e-4 * r[-1, 1]
    # a frozen step must use the weights' own S and P (their buffers are sized for them)
    prm2 = M.LadmmParams(lam=1e-2, rho=1.0, gamma=1.0 / 0.3321609, S=S + 2, P=P, h=0.05,
                         freeze_after=k0, iters=iters)
    with pytest.raises(M.api._lib.DsnlmError):
        M.ladmm_step(op, prm2, iters + 1, w, x2, v2, u2)


@pytest.mark.parametrize("n1,n2,iters", [(33, 29, 4), (37, 130, 3), (70, 64, 2), (9, 11, 2), (16, 65, 5), (512, 512, 2)])
def test_solve_one_launch_xstep_equals_two_launch_steps(n1, n2, iters):
    """The solve's x-steps for the 9-tap, factor-2 mirrored operator (tiles
    of 8 x 64 with their own residual window in LDS, x alternating between
    two buffers; after the first iteration each x-step is taken by the
    previous iteration's last kernel, the gather or the epilogue) give the
    same bits as the in-place two-launch step of ladmm_step, on shapes with
    ragged tiles, odd sizes, a single tile and odd and even iteration counts."""
    M = _M()
    print(f"one-launch x-step {n1}x{n2} iters={iters}", flush=True)
    rng = np.random.default_rng(n1 * 131 + n2)
    y = rng.uniform(0, 1, ((n1 + 1) // 2, (n2 + 1) // 2)).astype(np.float32)
    x0 = rng.uniform(0, 1, (n1, n2)).astype(np.float32)
    op = _sr_op(M, n1, n2, y=_t(y))
    prm = M.LadmmParams(lam=1e-2, rho=1.0, gamma=1.0 / 0.3321609, S=3, P=1, h=0.2,
                        freeze_after=1, iters=iters)
    x1, v1, u1 = _t(x0), _t(x0), torch.zeros((n1, n2), device="cuda")
    M.ladmm_solve(op, prm, x1, v1, u1)
    x2, v2, u2 = _t(x0), _t(x0), torch.zeros((n1, n2), device="cuda")
    w = None
    for k in range(1, iters + 1):
        w = M.ladmm_step(op, prm, k, w, x2, v2, u2)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and torch.equal(v1, v2) and torch.equal(u1, u2)
    # the same solve with residuals (another cached graph): the same iterates
    x3, v3, u3 = _t(x0), _t(x0), torch.zeros((n1, n2), device="cuda")
    res = torch.zeros((iters, 2), device="cuda")
    M.ladmm_solve(op, prm, x3, v3, u3, residuals=res)
    torch.cuda.synchronize()
    assert torch.equal(x1, x3) and torch.equal(v1, v3) and torch.equal(u1, u3)
    assert bool(torch.isfinite(res).all())


def test_frozen_weights_converge_to_fixed_point():
    """16x16 super-resolution with weights frozen after the first iteration
    and an inactive box: the iterates reach the solution of
    (W A^T A + rho (I - W)) x = W A^T y with W = W(z_1) (oracle, FP64)."""
    M = _M()
    n, S, P, h, rho = 16, 3, 1, 0.1, 1.0
    clean, _ = synth.piecewise_smooth(n, n, 7, 0.0)
    rng = np.random.default_rng(3)
    taps32 = TAPS.astype(np.float32)
    y = (L.sr_forward(clean, taps32, 2) + 0.01 * rng.standard_normal((8, 8))).astype(np.float32)
    x0 = np.full((n, n), 0.5, np.float32)
    A = L.sr_dense((n, n), taps32, 2, "symmetric")
    gamma = np.float32(1.0 / np.linalg.norm(A, 2) ** 2)
    alpha = 1.0 / float(gamma)
    grad_f = lambda v: L.sr_adjoint(L.sr_forward(v, taps32, 2) - y, taps32, 2, v.shape)
    # oracle: first iteration gives the guide z_1 = x_1 + u_0 = x_1
    x1 = np.clip((alpha * x0 + rho * (x0 - 0) - grad_f(x0)) / (alpha + rho), -10, 10)
    W = R.dense_weights(x1, S, P, h)["W"]
    xs = np.linalg.solve(W @ A.T @ A + rho * (np.eye(n * n) - W), W @ A.T @ y.ravel().astype(np.float64))
    op = _sr_op(M, n, n, y=_t(y))
    prm = M.LadmmParams(lam=1e-2, rho=rho, gamma=float(gamma), S=S, P=P, h=h, freeze_after=1,
                        iters=2500, lo=-10.0, hi=10.0)
    x, v, u = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    with torch.cuda.stream(torch.cuda.Stream()):
        M.ladmm_solve(op, prm, x, v, u)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy().ravel() - xs).max() <= 2e-4
    assert np.abs((x - v).cpu().numpy()).max() <= 1e-5


def test_full_config_sr_solve_properties():
    """2x super-resolution at 512x512 (S = 10, P = 3, 50 iterations, weights
    frozen after 5): finite residuals, iterates inside the box, the frozen
    phase's primal residual decreasing, and the first iteration equal to the
    oracle on sampled rows of the x-step."""
    M = _M()
    cfg = synth.config1_inputs(512)
    n = 512
    taps32 = TAPS.astype(np.float32)
    op = _sr_op(M, n, n, y=None)
    xc = _t(cfg["clean"])
    y = M.ladmm_apply_forward(op, xc) + _t(cfg["lr_noise"])
    op.y = y
    x0 = synth.bicubic_upsample(y.cpu().numpy(), 2)
    gamma = 1.0 / M.ladmm_operator_norm2(op, 300)
    prm = M.LadmmParams(lam=cfg["lam"], rho=cfg["rho"], gamma=gamma, S=10, P=3, h=cfg["h"],
                        freeze_after=5, iters=50)
    x, v, u = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    res = torch.zeros((50, 2), device="cuda")
    print("SR 512x512 solve, 50 iterations", flush=True)
    with torch.cuda.stream(torch.cuda.Stream()):
        M.ladmm_solve(op, prm, x, v, u, residuals=res)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    assert np.all(np.isfinite(r))
    assert float(x.min()) >= 0.0 and float(x.max()) <= 1.0
    assert r[-1, 0] < r[6, 0]
    # reconstruction is closer to the ground truth than the initialisation
    err0 = float(np.sqrt(np.mean((x0 - cfg["clean"]) ** 2)))
    err = float(torch.sqrt(torch.mean((x - xc) ** 2)))
    assert err < err0


@pytest.mark.parametrize("k0,steps", [(1, 3), (2, 4)])
def test_standard_admm_cg_matches_oracle(k0, steps):
    """Standard ADMM (CG inversion, 8 CG steps) from the same start: every
    iterate against the FP64 oracle run for the same number of outer steps."""
    M = _M()
    n, S, P, cg = 32, 3, 1, 8
    clean, y, x0 = _sr_problem(n, 41, S, P)
    lam, rho = np.float32(1e-2), np.float32(1.0)
    h = float(np.float32(math.sqrt(lam / rho)))
    taps32 = TAPS.astype(np.float32)
    op = _sr_op(M, n, n, y=_t(y))
    prm = M.LadmmParams(lam=float(lam), rho=float(rho), gamma=1.0, S=S, P=P, freeze_after=k0, iters=steps)
    x, v, u = _t(x0), _t(x0), torch.zeros((n, n), device="cuda")
    res = torch.zeros((steps, 2), device="cuda")
    M.admm_cg_solve(op, prm, cg, x, v, u, residuals=res)
    out = L.admm_cg(x0, y, taps32, 2, rho=float(rho), S=S, P=P, h=h, iters=steps, freeze_after=k0,
                    cg_iters=cg, v0=x0, u0=np.zeros_like(x0))
    tol = 1e-4 * steps
    assert np.abs(x.cpu().numpy() - out["x"]).max() <= tol
    assert np.abs(v.cpu().numpy() - out["v"]).max() <= tol
    assert np.abs(u.cpu().numpy() - out["u"]).max() <= tol
    r = res.cpu().numpy()
    assert np.all(np.isfinite(r))
    assert np.abs(r[-1] - out["residuals"][-1]).max() <= 1e-4
