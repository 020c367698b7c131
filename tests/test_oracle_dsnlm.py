"""CPU pins for the FP64 DSG-NLM oracle (no GPU).

Each test checks the oracle against something other than itself: a second
independent coding of the same definition, the properties the cited theorem
fixes (Section 3: W symmetric, doubly stochastic, eigenvalues in [0, 1]),
closed forms for special guides, or library constructions.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

import synth
from oracle import dsnlm_ref as R

SHAPES = [
    # (n1, n2, S, P): tiny shapes incl. S >= size, P >= S, one-row images
    (7, 6, 2, 1),
    (6, 7, 3, 2),
    (5, 5, 1, 3),
    (4, 4, 6, 1),
    (1, 6, 2, 0),
    (6, 1, 3, 0),
    (3, 8, 0, 1),
]


def _img(n1, n2, seed):
    _, noisy = synth.piecewise_smooth(n1, n2, seed, 0.05)
    return noisy


@pytest.mark.parametrize("n1,n2,S,P", SHAPES)
def test_two_routes_agree(n1, n2, S, P):
    """The dense matrices of S1-S3 (patches from numpy's symmetric padding)
    and the band-by-band route (its own mirror indexing) agree."""
    z = _img(n1, n2, 11)
    x = _img(n1, n2, 12)
    h = 0.08
    yd = R.dsnlm_dense(x, z, S, P, h)
    ys = R.dsnlm_shifts(x, z, S, P, h)["y"].numpy()
    assert np.abs(yd - ys).max() <= 1e-13
    dw = R.dense_weights(z, S, P, h)
    sh = R.dsnlm_shifts(x, z, S, P, h, want="weights")
    assert np.abs(dw["omega"] - sh["omega"].numpy().ravel()).max() <= 1e-12
    assert np.abs(dw["delta"] - sh["delta"].numpy().ravel()).max() <= 1e-13
    assert abs(dw["m"] - float(sh["m"])) <= 1e-13


@pytest.mark.parametrize("n1,n2,S,P,h", [(7, 6, 2, 1, 0.1), (8, 8, 3, 1, 0.05), (6, 9, 4, 2, 0.3)])
def test_theorem_properties(n1, n2, S, P, h):
    """W symmetric, nonnegative, rows/columns sum to 1, spectrum in (0, 1]
    with the constant vector as top eigenvector."""
    z = _img(n1, n2, 21)
    W = R.dense_weights(z, S, P, h)["W"]
    n = n1 * n2
    assert np.abs(W - W.T).max() <= 1e-15
    assert W.min() >= 0.0
    assert np.abs(W.sum(0) - 1).max() <= 1e-12
    assert np.abs(W.sum(1) - 1).max() <= 1e-12
    ev, V = np.linalg.eigh(W)
    assert ev[0] > 0.0
    assert ev[-1] <= 1 + 1e-12 and abs(ev[-1] - 1) <= 1e-12
    top = V[:, -1] * np.sign(V[0, -1])
    assert np.abs(top - 1 / math.sqrt(n)).max() <= 1e-8


def test_invariants_medium():
    """Constants are fixed points for any guide; the image mean is preserved;
    the output stays within [min x, max x]."""
    z = _img(24, 19, 31)
    x = _img(24, 19, 32)
    S, P, h = 4, 2, 0.07
    y = R.dsnlm_shifts(x, z, S, P, h)["y"].numpy()
    c = R.dsnlm_shifts(np.full(x.shape, 0.37), z, S, P, h)["y"].numpy()
    assert np.abs(c - 0.37).max() <= 1e-15
    assert abs(y.sum() - x.astype(np.float64).sum()) <= 1e-11
    assert y.min() >= x.min() - 1e-14 and y.max() <= x.max() + 1e-14


def test_vanishing_bandwidth_is_identity():
    """h -> 0 with all patches distinct: every off-diagonal weight underflows,
    W = I and y equals x bit for bit."""
    rng = np.random.default_rng(5)
    z = rng.uniform(0, 1, size=(9, 10)).astype(np.float32)
    x = rng.uniform(0, 1, size=(9, 10)).astype(np.float32)
    out = R.dsnlm_shifts(x, z, 3, 1, 1e-6)
    assert np.array_equal(out["y"].numpy(), x.astype(np.float64))
    assert float(out["m"]) == 1.0


def test_constant_guide_closed_form_max():
    """Constant guide, S = 1: the weights are the hat alone, separable across
    axes, and the largest row sum after S2 is (3/4 + 1/(2 sqrt 3))^2
    (attained one pixel in from a corner, for n1, n2 >= 4)."""
    for n1, n2 in [(4, 4), (6, 5), (9, 12)]:
        z = np.full((n1, n2), 0.3)
        dw = R.dense_weights(z, 1, 1, 0.1)
        expect = (0.75 + 1.0 / (2.0 * math.sqrt(3.0))) ** 2
        assert abs(dw["m"] - expect) <= 1e-15
        sh = R.dsnlm_shifts(z, z, 1, 1, 0.1, want="weights")
        assert abs(float(sh["m"]) - expect) <= 1e-15


@pytest.mark.parametrize("S", [1, 2, 3])
def test_constant_guide_kron_toeplitz(S):
    """Constant guide: W1 is the Kronecker product of two 1-D Toeplitz hat
    matrices (row-major pixel order), and interior row sums equal (S+1)^2."""
    n1, n2 = 9, 11
    z = np.full((n1, n2), 0.6)
    dw = R.dense_weights(z, S, 1, 0.2)

    def toep(n):
        col = np.array([max(0.0, 1 - k / (S + 1.0)) if k <= S else 0.0 for k in range(n)])
        return scipy.linalg.toeplitz(col)

    assert np.abs(dw["W1"] - np.kron(toep(n1), toep(n2))).max() <= 1e-15
    om = dw["omega"].reshape(n1, n2)
    assert np.abs(om[S:n1 - S, S:n2 - S] - (S + 1) ** 2).max() <= 1e-12


@pytest.mark.parametrize("P", [0, 1, 2])
def test_kernel_normalisation_on_stripes(P):
    """Guide with rows alternating 0/1: every interior patch differs from the
    one a row below in all N_p^2 pixels by exactly 1, so D = N_p^2 and the
    kernel is exp(-1/(2h^2)) whatever the patch size (pins the N_p^2 h^2
    normalisation of eq. NLM)."""
    n1, n2, S, h = 12, 10, 2, 0.7
    z = np.tile((np.arange(n1) % 2)[:, None], (1, n2)).astype(np.float64)
    dw = R.dense_weights(z, S, P, h)
    lam = (1 - 1 / (S + 1.0))
    for i in range(P + 1, n1 - P - 2):
        for j in range(P, n2 - P):
            s = i * n2 + j
            r = (i + 1) * n2 + j
            assert abs(dw["W1"][s, r] - lam * math.exp(-1 / (2 * h * h))) <= 1e-15
            r2 = (i + 2) * n2 + j if i + 2 < n1 - P else None
            if r2 is not None:
                assert abs(dw["W1"][s, r2] - (1 - 2 / (S + 1.0))) <= 1e-15


def test_scale_invariance():
    """W(c z, c h) = W(z, h): the kernel depends on D/h^2 only."""
    z = _img(8, 7, 41)
    a = R.dense_weights(z, 2, 1, 0.1)["W"]
    b = R.dense_weights(3.0 * z.astype(np.float64), 2, 1, 0.3)["W"]
    assert np.abs(a - b).max() <= 1e-13


def test_mirror_index_matches_numpy_symmetric_pad():
    for n, P in [(5, 0), (5, 3), (7, 6), (1, 0)]:
        a = np.arange(n, dtype=np.float64)
        assert np.array_equal(a[R.sym_index(n, P)], np.pad(a, P, mode="symmetric"))


def test_argument_domain():
    z = np.zeros((4, 4))
    with pytest.raises(ValueError):
        R.check_args(4, 4, 1, 4, 0.1)
    with pytest.raises(ValueError):
        R.check_args(4, 4, -1, 1, 0.1)
    with pytest.raises(ValueError):
        R.check_args(4, 4, 1, 1, 0.0)
    with pytest.raises(ValueError):
        R.check_args(4, 4, 1, 1, float("nan"))
    with pytest.raises(ValueError):
        R.dsnlm_shifts(z, z, 1, 1, -1.0)


# ---- plain NLM (eq. NLM) -------------------------------------------------
def test_nlm_two_routes_agree_and_rows_are_stochastic():
    _, z = synth.piecewise_smooth(7, 9, 61, 0.05)
    _, x = synth.piecewise_smooth(7, 9, 62, 0.05)
    S, P, h = 2, 1, 0.1
    y1 = R.nlm_dense(x, z, S, P, h)
    y2 = R.nlm_shifts(x, z, S, P, h)
    assert np.abs(y1 - y2).max() <= 1e-13
    K = R.dense_weights(z, S, P, h)["K"]
    Kn = K / K.sum(1, keepdims=True)
    assert np.abs(Kn.sum(1) - 1).max() <= 1e-14
    assert np.abs(R.nlm_dense(np.full((7, 9), 0.3), z, S, P, h) - 0.3).max() <= 1e-14
    assert y1.min() >= x.min() - 1e-15 and y1.max() <= x.max() + 1e-15


def test_nlm_large_bandwidth_is_the_window_mean():
    """h -> infinity: k = 1 on the (border-cut) window, so y_s is the plain mean
    of x over Omega_s, a box filter computed here with numpy slicing."""
    _, x = synth.piecewise_smooth(8, 11, 63, 0.05)
    x = x.astype(np.float64)
    S, P = 2, 1
    y = R.nlm_dense(x, x, S, P, 1e9)
    n1, n2 = x.shape
    ref = np.empty_like(y)
    for i in range(n1):
        for j in range(n2):
            blk = x[max(0, i - S):min(n1, i + S + 1), max(0, j - S):min(n2, j + S + 1)]
            ref[i, j] = blk.mean()
    assert np.abs(y - ref).max() <= 1e-12


def test_nlm_vanishing_bandwidth_is_identity():
    rng = np.random.default_rng(64)
    z = rng.random((6, 7))
    x = rng.random((6, 7))
    y = R.nlm_dense(x, z, 2, 1, 1e-4)
    assert np.array_equal(y, x.astype(np.float64))


@pytest.mark.parametrize("n1,n2,S,P", SHAPES + [(9, 13, 3, 4)])
def test_integral_image_distances_equal_direct_sums(n1, n2, S, P):
    """The fast scheme of Section 3 (integral image of the squared-difference
    image per shift, four lookups per patch) against the direct N_p^2 sums.
    On a guide quantised to multiples of 2^-8 every partial sum is exact in
    FP64, so the distances, and with them every output, agree bit for bit;
    on an unquantised guide they agree to rounding."""
    zq = np.round(_img(n1, n2, 13) * 256.0) / 256.0
    x = _img(n1, n2, 14)
    h = 0.1
    a = R.dsnlm_shifts(x, zq, S, P, h)
    b = R.dsnlm_shifts(x, zq, S, P, h, distances="integral")
    assert torch.equal(a["y"], b["y"]) and torch.equal(a["delta"], b["delta"])
    z = _img(n1, n2, 15)
    a = R.dsnlm_shifts(x, z, S, P, h)["y"]
    b = R.dsnlm_shifts(x, z, S, P, h, distances="integral")["y"]
    assert float((a - b).abs().max()) <= 1e-12


@pytest.mark.parametrize("n1,n2,S,P", [(7, 9, 3, 1), (6, 5, 6, 2), (1, 8, 2, 0)])
def test_pixel_rows_equal_dense_matrices(n1, n2, S, P):
    """The one-pixel-at-a-time route against the n x n matrices of steps
    S1-S3 built literally, at every pixel of a tiny image (windows cut by
    every border, S beyond the image)."""
    z, x = _img(n1, n2, 31), _img(n1, n2, 32)
    h = 0.15
    dw = R.dense_weights(z, S, P, h)
    pix = [(i, j) for i in range(n1) for j in range(n2)]
    q = R.dsnlm_pixels(x, z, S, P, h, pix, dw["m"])
    y = (dw["W"] @ x.astype(np.float64).ravel())
    assert np.abs(q["omega"] - dw["omega"]).max() <= 1e-13
    assert np.abs(q["delta"] - dw["delta"]).max() <= 1e-13
    assert np.abs(q["y"] - y).max() <= 1e-13


def test_pixel_rows_equal_shift_bands():
    """The same against the band-by-band route on a larger image, at the
    corners, edges, an interior pixel and the maximising pixel."""
    n1, n2, S, P, h = 40, 57, 10, 3, 0.08
    z, x = _img(n1, n2, 33), _img(n1, n2, 34)
    o = R.dsnlm_shifts(x, z, S, P, h)
    am = o["argmax"]
    pix = [(0, 0), (0, n2 - 1), (n1 - 1, 0), (n1 - 1, n2 - 1), (3, 20), (20, 2), (17, 31),
           (am // n2, am % n2)]
    q = R.dsnlm_pixels(x, z, S, P, h, pix, float(o["m"]))
    for k, (i, j) in enumerate(pix):
        assert abs(q["omega"][k] - float(o["omega"][i, j])) <= 1e-12
        assert abs(q["delta"][k] - float(o["delta"][i, j])) <= 1e-12
        assert abs(q["y"][k] - float(o["y"][i, j])) <= 1e-12
    assert q["delta"][-1] == pytest.approx(float(o["m"]), abs=1e-12)
