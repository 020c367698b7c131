"""FP64 oracle for the doubly stochastic NLM denoiser (DSG-NLM).

TEST INFRASTRUCTURE ONLY -- imported by tests/, the smoke check and the bench's
CPU-baseline leg; never by the HIP library.

What is computed (Section 3 of the paper):

* patches P_s of side N_p = 2P+1 centred at each pixel s (eq. NLM); pixels of
  a patch that fall outside the image take the half-sample symmetric mirror of
  the guide (index -1 -> 0, n -> n-1; the paper does not say how patches
  at the border are formed);
* kernel k_{s,r} = exp(-||P_s - P_r||^2 / (2 N_p^2 h^2)) for r in the search
  window Omega_s = {r in the image : ||r - s||_inf <= S}; the window is cut at
  the image border and includes r = s (eq. NLM, with the bandwidth h in
  place of the paper's sigma);
* step S1: w = Lambda_{s,r} k_{s,r}, Lambda the separable hat with argument
  (s - r)/(S + 1);
* step S2: w <- w (row sum_s)^(-1/2) (column sum_r)^(-1/2);
* step S3: with m the largest row sum after S2, w <- w/m and then the diagonal
  w_ss <- 1 + w_ss - sum_r w_sr (the sum includes the diagonal term, which
  makes every row sum exactly one);
* output W x.  Algorithm 2 computes the same product without storing W.

Three routes are provided:

dense_weights / dsnlm_dense -- build the n x n matrices of eqs. S1-S3 literally
                               (tiny images only; patches cut from numpy's
                               symmetric padding);
dsnlm_shifts                -- the same matrices evaluated one window shift at
                               a time: for a shift d the entries (s, s+d) of
                               every matrix form one band, computed for all
                               pixels s at once (torch CPU float64,
                               differentiable), with the patch distances summed
                               directly over the N_p^2 patch offsets (no
                               box-sum trick) and the mirror indexing of
                               sym_index.  This is the route used for GPU
                               parity and for the CPU baseline.
dsnlm_pixels                -- the rows of the same matrices at chosen
                               pixels only (numpy float64), for images the
                               band route cannot afford: omega at a pixel and
                               at each of its partners from their own rows,
                               delta and y at the pixel given the image's m.
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = [
    "sym_index",
    "pad_symmetric",
    "hat",
    "dense_weights",
    "dsnlm_dense",
    "dsnlm_shifts",
    "dsnlm_pixels",
    "check_args",
]


def check_args(n1: int, n2: int, S: int, P: int, h: float) -> None:
    """Input domain: S >= 0, P >= 0, P < min(n1, n2) (one mirror reflection
    suffices), h finite and > 0."""
    if n1 < 1 or n2 < 1:
        raise ValueError("empty image")
    if S < 0 or P < 0:
        raise ValueError("S and P must be >= 0")
    if P >= min(n1, n2):
        raise ValueError("P must be < min(n1, n2)")
    if not (math.isfinite(float(h)) and float(h) > 0):
        raise ValueError("h must be finite and > 0")


def sym_index(n: int, P: int) -> np.ndarray:
    """Indices into [0, n) for padded positions -P .. n+P-1 under the
    half-sample symmetric mirror (-1 -> 0, -2 -> 1, n -> n-1)."""
    k = np.arange(-P, n + P)
    k = np.where(k < 0, -k - 1, k)
    k = np.where(k >= n, 2 * n - 1 - k, k)
    return k


def pad_symmetric(z: np.ndarray, P: int) -> np.ndarray:
    """Mirror-pad by P on every side (numpy's 'symmetric' mode)."""
    return np.pad(np.asarray(z, dtype=np.float64), P, mode="symmetric")


def hat(d: int, S: int) -> float:
    """One factor of the separable hat Lambda of step S1 at offset d."""
    return 1.0 - abs(d) / (S + 1.0)


# ---------------------------------------------------------------------------
# Route 1: the matrices of eqs. S1-S3, built densely.
# ---------------------------------------------------------------------------
def dense_weights(z, S: int, P: int, h: float) -> dict:
    """Return the intermediate and final matrices of steps S1-S3 for guide z.

    Keys: K (kernel, zero outside the windows), Lam (hat), W1 (after S1),
    W2 (after S2), W (after S3), omega (row sums of W1), delta (row sums of
    W2), m (max of delta).  Pixel s = (i, j) has index i*n2 + j.
    """
    z = np.asarray(z, dtype=np.float64)
    n1, n2 = z.shape
    check_args(n1, n2, S, P, h)
    Np = 2 * P + 1
    zp = pad_symmetric(z, P)
    n = n1 * n2
    patches = np.empty((n, Np * Np))
    for i in range(n1):
        for j in range(n2):
            patches[i * n2 + j] = zp[i:i + Np, j:j + Np].ravel()
    ii = np.repeat(np.arange(n1), n2)
    jj = np.tile(np.arange(n2), n1)
    di = ii[:, None] - ii[None, :]
    dj = jj[:, None] - jj[None, :]
    inwin = (np.abs(di) <= S) & (np.abs(dj) <= S)
    rows, cols = np.nonzero(inwin)
    dist = np.zeros((n, n))
    dist[rows, cols] = ((patches[rows] - patches[cols]) ** 2).sum(1)
    K = np.where(inwin, np.exp(-dist / (2.0 * Np * Np * h * h)), 0.0)
    Lam = np.where(inwin, (1.0 - np.abs(di) / (S + 1.0)) * (1.0 - np.abs(dj) / (S + 1.0)), 0.0)
    W1 = Lam * K
    rowsum = W1.sum(1)
    colsum = W1.sum(0)
    W2 = W1 * rowsum[:, None] ** -0.5 * colsum[None, :] ** -0.5
    delta = W2.sum(1)
    m = delta.max()
    W = W2 / m
    full = W.sum(1)
    W[np.arange(n), np.arange(n)] = 1.0 + np.diag(W) - full
    return dict(K=K, Lam=Lam, W1=W1, W2=W2, W=W, omega=rowsum, delta=delta, m=m)


def dsnlm_dense(x, z, S: int, P: int, h: float) -> np.ndarray:
    """y = W(z) x via the dense matrix of step S3 (tiny images only)."""
    x = np.asarray(x, dtype=np.float64)
    W = dense_weights(z, S, P, h)["W"]
    return (W @ x.ravel()).reshape(x.shape)


# ---------------------------------------------------------------------------
# Route 2: the matrices of S1-S3 band by band (one band per window shift).
# ---------------------------------------------------------------------------
def _as_t(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(torch.float64)
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def _shift_ranges(n: int, d: int):
    """Pixels s with s + d inside [0, n): the half-open range [lo, hi)."""
    return max(0, -d), min(n, n - d)


def integral_distances(zp: torch.Tensor, i0: int, i1: int, j0: int, j1: int, dy: int, dx: int,
                       Np: int) -> torch.Tensor:
    """Patch distances of the pixels s in [i0, i1) x [j0, j1) to s + d from
    the integral image of the squared-difference image of the shift (Section
    3, the fast scheme after Algorithm 2): e(p) = (z(p) - z(p + d))^2 over the
    padded rows and columns the patches cover, I = its 2-D prefix sums with a
    zero first row and column, and each distance a box of I read at its four
    corners.  zp: the guide padded by P (padded index = image index + P)."""
    a = zp[i0:i1 + Np - 1, j0:j1 + Np - 1]
    b = zp[i0 + dy:i1 + dy + Np - 1, j0 + dx:j1 + dx + Np - 1]
    e = (a - b) ** 2
    integ = torch.zeros((e.shape[0] + 1, e.shape[1] + 1), dtype=torch.float64)
    integ[1:, 1:] = torch.cumsum(torch.cumsum(e, dim=0), dim=1)
    h1, w1 = i1 - i0, j1 - j0
    return (integ[Np:Np + h1, Np:Np + w1] - integ[0:h1, Np:Np + w1]
            - integ[Np:Np + h1, 0:w1] + integ[0:h1, 0:w1])


def dsnlm_shifts(x, z, S: int, P: int, h, want: str = "y", distances: str = "direct") -> dict:
    """y = W(z) x from the matrices of steps S1-S3, one window shift at a time
    (torch FP64).

    For a shift d = (dy, dx) the entries (s, s + d) of Lambda*K form one band
    of the matrix; it is computed for every pixel s at once.  The row sums of
    step S1 (omega), of step S2 (delta) and the product with the matrix of
    step S3 are accumulated band by band.
    x, z: 2-D arrays or tensors (cast to float64; autograd flows through them
    and through h when they are tensors that require grad).
    distances: "direct" sums every patch distance over its N_p^2 offsets (the
    brute force); "integral" reads it from the shift's integral image.
    Returns a dict with y (= W x), omega (row sums after S1), delta (row sums
    after S2), m (their maximum), argmax (flat index of the first maximal delta,
    which is where the derivative of the max is routed; the paper does not
    differentiate, so ties are broken towards the lowest index).
    """
    xt = _as_t(x)
    zt = _as_t(z)
    ht = h if isinstance(h, torch.Tensor) else torch.tensor(float(h), dtype=torch.float64)
    n1, n2 = zt.shape
    check_args(n1, n2, S, P, float(ht.detach()))
    Np = 2 * P + 1
    ri = torch.as_tensor(sym_index(n1, P))
    ci = torch.as_tensor(sym_index(n2, P))
    zp = zt[ri][:, ci]
    kappa = 1.0 / (2.0 * Np * Np * ht * ht)

    def weight(dy, dx):
        """Lambda_d * k_{s, s+d} on the pixels s with s + d in the image."""
        i0, i1 = _shift_ranges(n1, dy)
        j0, j1 = _shift_ranges(n2, dx)
        if i0 >= i1 or j0 >= j1:
            return None
        if distances == "integral":
            D = integral_distances(zp, i0, i1, j0, j1, dy, dx, Np)
        else:
            D = torch.zeros((i1 - i0, j1 - j0), dtype=torch.float64)
            for ty in range(Np):
                for tx in range(Np):
                    a = zp[i0 + ty:i1 + ty, j0 + tx:j1 + tx]
                    b = zp[i0 + dy + ty:i1 + dy + ty, j0 + dx + tx:j1 + dx + tx]
                    D = D + (a - b) ** 2
        lam = hat(dy, S) * hat(dx, S)
        return (i0, i1, j0, j1), lam * torch.exp(-kappa * D)

    shifts = [(dy, dx) for dy in range(-S, S + 1) for dx in range(-S, S + 1)]

    # step S1 row sums: omega_s = sum_r Lambda k
    omega = torch.zeros((n1, n2), dtype=torch.float64)
    for dy, dx in shifts:
        wres = weight(dy, dx)
        if wres is None:
            continue
        (i0, i1, j0, j1), a = wres
        omega[i0:i1, j0:j1] += a
    # step S2 (column sums equal row sums by symmetry): delta_s = sum_r (omega_s omega_r)^-1/2 Lambda k
    delta = torch.zeros((n1, n2), dtype=torch.float64)
    for dy, dx in shifts:
        wres = weight(dy, dx)
        if wres is None:
            continue
        (i0, i1, j0, j1), a = wres
        gs = omega[i0:i1, j0:j1]
        gr = omega[i0 + dy:i1 + dy, j0 + dx:j1 + dx]
        delta[i0:i1, j0:j1] += (gs * gr) ** -0.5 * a
    flat = delta.reshape(-1)
    am = int(torch.argmax(flat.detach()))
    m = flat[am]
    out = dict(omega=omega, delta=delta, m=m, argmax=am)
    if want == "weights":
        return out
    # step S3: off-diagonal w = m^-1 (omega_s omega_r)^-1/2 Lambda k, diagonal 1 minus the rest of
    # the row, so (W x)_s = sum_r w x_r + (1 - sum_r w) x_s with r = s inside both sums
    acc = torch.zeros((n1, n2), dtype=torch.float64)
    hs = torch.zeros((n1, n2), dtype=torch.float64)
    for dy, dx in shifts:
        wres = weight(dy, dx)
        if wres is None:
            continue
        (i0, i1, j0, j1), a = wres
        gs = omega[i0:i1, j0:j1]
        gr = omega[i0 + dy:i1 + dy, j0 + dx:j1 + dx]
        w = (gs * gr) ** -0.5 * a / m
        acc[i0:i1, j0:j1] += w * xt[i0 + dy:i1 + dy, j0 + dx:j1 + dx]
        hs[i0:i1, j0:j1] += w
    out["y"] = acc + (1.0 - hs) * xt
    return out


# ---------------------------------------------------------------------------
# Route 3: the rows of S1-S3 one pixel at a time (images of any size).
# ---------------------------------------------------------------------------
def _row_weights(zp: np.ndarray, n1: int, n2: int, ci, cj, S: int, P: int, kappa: float):
    """Step S1 rows of the pixels (ci[k], cj[k]): for each, the partners
    r = (ci + dy, cj + dx) of its window, a mask of those inside the image, and
    their weights Lambda_d k_{s,r} (zero outside), the patch distances summed
    directly over the N_p^2 offsets of the guide padded by P (zp).  Arrays of
    shape (len(ci), (2S + 1)^2)."""
    Np = 2 * P + 1
    dy, dx = np.meshgrid(np.arange(-S, S + 1), np.arange(-S, S + 1), indexing="ij")
    ci = np.asarray(ci)[:, None]
    cj = np.asarray(cj)[:, None]
    ri, rj = ci + dy.ravel()[None, :], cj + dx.ravel()[None, :]
    keep = (ri >= 0) & (ri < n1) & (rj >= 0) & (rj < n2)
    qi, qj = np.where(keep, ri, ci), np.where(keep, rj, cj)  # in range; masked below
    dist = np.zeros(ri.shape)
    for ty in range(Np):
        for tx in range(Np):
            dist += (zp[ci + ty, cj + tx] - zp[qi + ty, qj + tx]) ** 2
    lam = (1.0 - np.abs(dy.ravel()) / (S + 1.0)) * (1.0 - np.abs(dx.ravel()) / (S + 1.0))
    return ri, rj, keep, np.where(keep, lam[None, :] * np.exp(-kappa * dist), 0.0)


def dsnlm_pixels(x, z, S: int, P: int, h: float, pixels, m: float) -> dict:
    """omega, delta and y = (W x) at the listed pixels, each from its own rows
    of the matrices of steps S1-S3, for images too large for the band route.

    omega_s is the row sum of step S1 at s; delta_s = sum_r (omega_s
    omega_r)^-1/2 w1_{s,r} (step S2, which needs omega at every partner r of
    s, each from that partner's own row); y_s = sum_r w_{s,r} x_r + (1 -
    sum_r w_{s,r}) x_s with w = (omega_s omega_r)^-1/2 w1 / m (step S3).  The
    normalisation m, the maximum of delta over the whole image, is an input:
    the caller checks it separately (delta at the maximising pixel is one of
    the pixels this function can evaluate).
    pixels: iterable of (i, j).  Returns arrays omega, delta, y over them.
    """
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n1, n2 = z.shape
    check_args(n1, n2, S, P, h)
    Np = 2 * P + 1
    zp = z[sym_index(n1, P)][:, sym_index(n2, P)]
    kappa = 1.0 / (2.0 * Np * Np * h * h)
    om, de, ys = [], [], []
    for i, j in pixels:
        ri, rj, keep, w1 = _row_weights(zp, n1, n2, [i], [j], S, P, kappa)
        ri, rj, w1 = ri[0][keep[0]], rj[0][keep[0]], w1[0][keep[0]]
        om_s = w1.sum()
        om_r = _row_weights(zp, n1, n2, ri, rj, S, P, kappa)[3].sum(axis=1)
        w2 = (om_s * om_r) ** -0.5 * w1
        w = w2 / m
        om.append(om_s)
        de.append(w2.sum())
        ys.append((w * x[ri, rj]).sum() + (1.0 - w.sum()) * x[i, j])
    return dict(omega=np.array(om), delta=np.array(de), y=np.array(ys))


# ---------------------------------------------------------------------------
# Plain NLM (eq. NLM): the row-stochastic filter DSG-NLM is built from.
# ---------------------------------------------------------------------------
def nlm_dense(x, z, S: int, P: int, h: float) -> np.ndarray:
    """y = K x with K = diag(1 / sum_r k_{s,r}) [k_{s,r}]: eq. NLM written as a
    matrix (kernel of the guide z, no hat, window cut at the border; tiny
    images only)."""
    x = np.asarray(x, dtype=np.float64)
    K = dense_weights(z, S, P, h)["K"]
    Kn = K / K.sum(1, keepdims=True)
    return (Kn @ x.ravel()).reshape(x.shape)


def nlm_shifts(x, z, S: int, P: int, h: float) -> np.ndarray:
    """eq. NLM with the pixel loop vectorised and a Python loop over the
    (2S+1)^2 window shifts, patch distances summed directly (torch FP64):
    y_s = sum_r k_{s,r} x_r / sum_r k_{s,r}."""
    xt = _as_t(x)
    zt = _as_t(z)
    n1, n2 = zt.shape
    check_args(n1, n2, S, P, float(h))
    Np = 2 * P + 1
    zp = zt[torch.as_tensor(sym_index(n1, P))][:, torch.as_tensor(sym_index(n2, P))]
    kappa = 1.0 / (2.0 * Np * Np * float(h) ** 2)
    num = torch.zeros((n1, n2), dtype=torch.float64)
    den = torch.zeros((n1, n2), dtype=torch.float64)
    for dy in range(-S, S + 1):
        for dx in range(-S, S + 1):
            i0, i1 = _shift_ranges(n1, dy)
            j0, j1 = _shift_ranges(n2, dx)
            if i0 >= i1 or j0 >= j1:
                continue
            D = torch.zeros((i1 - i0, j1 - j0), dtype=torch.float64)
            for ty in range(Np):
                for tx in range(Np):
                    a = zp[i0 + ty:i1 + ty, j0 + tx:j1 + tx]
                    b = zp[i0 + dy + ty:i1 + dy + ty, j0 + dx + tx:j1 + dx + tx]
                    D = D + (a - b) ** 2
            k = torch.exp(-kappa * D)
            num[i0:i1, j0:j1] += k * xt[i0 + dy:i1 + dy, j0 + dx:j1 + dx]
            den[i0:i1, j0:j1] += k
    return (num / den).numpy()
