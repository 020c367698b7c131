// The super-resolution forward model of Section 4.1 on the device: A =
// decimation by a factor f after a separable blur with mirrored (boundary 0)
// or periodic (boundary 1) extension, its exact adjoint, and the linearized
// x-step of Algorithm 1 built on them.  Shared by the solver kernels and the
// gather of the frozen apply, which can finish an iteration with the next
// iteration's x-step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace dsnlm {

constexpr int kMaxTaps = 31;

struct Taps {
    float t[kMaxTaps];
};

struct SRGeom {
    int n1, n2;   // high-resolution size
    int m1, m2;   // low-resolution size, ceil(n / factor)
    int f;        // decimation factor
    int bs;       // blur size (odd)
    int R;        // (bs - 1) / 2
};

// Source index in [0, n) of padded position k (|k| < 2n).
template <int BOUNDARY>
__device__ __forceinline__ int src_index(int k, int n) {
    if (BOUNDARY == 0) {
        if (k < 0) return -k - 1;
        if (k >= n) return 2 * n - 1 - k;
        return k;
    }
    if (k < 0) return k + n;
    if (k >= n) return k - n;
    return k;
}

// The padded positions that map onto pixel i (itself and up to two copies).
template <int BOUNDARY>
__device__ __forceinline__ int preimages(int i, int n, int R, int* out) {
    int c = 0;
    out[c++] = i;
    if (BOUNDARY == 0) {
        if (i <= R - 1) out[c++] = -1 - i;
        if (i >= n - R) out[c++] = 2 * n - 1 - i;
    } else {
        if (i <= R - 1) out[c++] = i + n;
        if (i >= n - R) out[c++] = i - n;
    }
    return c;
}

// The low-resolution samples I = lo..hi whose blur footprint covers padded
// position p: 0 <= p - f I + R <= bs - 1, clamped to the grid [0, m).
__device__ __forceinline__ void footprint(int p, int f, int R, int bs, int m, int* lo, int* hi) {
    int l = p + R - (bs - 1);
    l = l <= 0 ? 0 : (l + f - 1) / f;
    int h = p + R;
    h = h < 0 ? -1 : h / f;
    *lo = l;
    *hi = h > m - 1 ? m - 1 : h;
}

// (A^T r)(i, j): gather over the low-resolution samples whose footprint covers
// a preimage of (i, j).  BS > 0: blur size BS and factor F fixed at compile
// time, with at most ceil(BS / F) samples per axis and preimage (loops
// unrolled, same order of additions as the general form).
// Readers of the low-resolution residual r(I, J): the whole grid in global
// memory, or a block's window of it in LDS.
struct RGlobal {
    const float* __restrict__ r;
    int m2;
    __device__ float operator()(int I, int J) const { return r[(size_t)I * m2 + J]; }
};
struct RLds {
    const float* r;
    int stride, I0, J0;
    __device__ float operator()(int I, int J) const { return r[(I - I0) * stride + (J - J0)]; }
};

template <int BOUNDARY, int BS, int F, class RD>
__device__ __forceinline__ float sr_adjoint_at(const RD& rd, int i, int j, const SRGeom& g, const Taps& taps) {
    constexpr int NS = BS > 0 ? (BS + F - 1) / F : 1;
    const int f = BS > 0 ? F : g.f, bs = BS > 0 ? BS : g.bs, R = (bs - 1) / 2;
    int pi[3], pj[3];
    const int ci = preimages<BOUNDARY>(i, g.n1, R, pi);
    const int cj = preimages<BOUNDARY>(j, g.n2, R, pj);
    float acc = 0.f;
    for (int a = 0; a < ci; ++a) {
        const int ip = pi[a];
        int Ilo, Ihi;
        footprint(ip, f, R, bs, g.m1, &Ilo, &Ihi);
        if constexpr (BS > 0) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const int I = Ilo + t;
                if (I <= Ihi) {
                    const float ta = taps.t[ip - F * I + R];
                    float rowacc = 0.f;
                    for (int b = 0; b < cj; ++b) {
                        const int jp = pj[b];
                        int Jlo, Jhi;
                        footprint(jp, F, R, BS, g.m2, &Jlo, &Jhi);
#pragma unroll
                        for (int q = 0; q < NS; ++q) {
                            const int J = Jlo + q;
                            if (J <= Jhi) rowacc = fmaf(taps.t[jp - F * J + R], rd(I, J), rowacc);
                        }
                    }
                    acc = fmaf(ta, rowacc, acc);
                }
            }
        } else {
            for (int I = Ilo; I <= Ihi; ++I) {
                const float ta = taps.t[ip - f * I + R];
                float rowacc = 0.f;
                for (int b = 0; b < cj; ++b) {
                    const int jp = pj[b];
                    int Jlo, Jhi;
                    footprint(jp, f, R, bs, g.m2, &Jlo, &Jhi);
                    for (int J = Jlo; J <= Jhi; ++J) rowacc = fmaf(taps.t[jp - f * J + R], rd(I, J), rowacc);
                }
                acc = fmaf(ta, rowacc, acc);
            }
        }
    }
    return acc;
}

struct StepScalars {
    float alpha, rho, mu, lo, hi;
};

// clip(mu (alpha x + rho (v - u) - grad)): the x-step at one pixel.
__device__ __forceinline__ float xstep_value(float grad, float x, float v, float u, const StepScalars& s) {
    const float xn = s.mu * (s.alpha * x + s.rho * (v - u) - grad);
    return fminf(fmaxf(xn, s.lo), s.hi);
}

// xo = the x-step and z = xo + u at idx.
__device__ __forceinline__ void xstep_store(float grad, const float* x, const float* v, const float* u, float* xo,
                                            float* z, size_t idx, const StepScalars& s) {
    const float uu = u[idx];
    const float xn = xstep_value(grad, x[idx], v[idx], uu, s);
    xo[idx] = xn;
    z[idx] = xn + uu;
}

// x <- clip(mu (alpha x + rho (v - u) - A^T r)); z = x + u.
// With step == 0 it only writes g = A^T r into xo (gradient / adjoint).
// Tap b[F t + ph] for a per-lane phase ph in [0, F) (0 past the kernel's end):
// every index is a compile-time constant, so the taps stay in scalar registers.
template <int BS, int F>
__device__ __forceinline__ float phase_tap(const Taps& taps, int t, int ph) {
    float v = taps.t[F * t];
#pragma unroll
    for (int e = 1; e < F; ++e)
        if (ph == e) v = F * t + e < BS ? taps.t[F * t + e] : 0.f;
    return v;
}

// (A^T r)(i, j) for a pixel with no mirrored or wrapped copy inside any
// footprint (R <= i < n1 - R, R <= j < n2 - R): the samples of an axis are
// I = (i + R) / F - t, t = 0 .. ceil(BS / F) - 1, with tap b[(i + R) % F + F t]
// (zero where that passes the kernel); they all lie inside the grid.
template <int BS, int F, class RD>
__device__ __forceinline__ float sr_adjoint_interior(const RD& rd, int i, int j, const Taps& taps) {
    constexpr int R = (BS - 1) / 2, NS = (BS + F - 1) / F;
    const int qi = i + R, qj = j + R;
    const int phi = qi % F, phj = qj % F;
    const int I0 = qi / F, J0 = qj / F;
    float tb[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) tb[q] = phase_tap<BS, F>(taps, q, phj);
    float rv[NS][NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int I = I0 - t > 0 ? I0 - t : 0;  // a zero tap's sample is clamped into the grid
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int J = J0 - q > 0 ? J0 - q : 0;
            rv[t][q] = rd(I, J);
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        float rowacc = 0.f;
#pragma unroll
        for (int q = 0; q < NS; ++q) rowacc = fmaf(tb[q], rv[t][q], rowacc);
        acc = fmaf(phase_tap<BS, F>(taps, t, phi), rowacc, acc);
    }
    return acc;
}

// The x-step of the 9-tap, factor-2 operator with mirrored boundary for a
// TH x TW tile of the high-resolution grid, by a block of NT threads.  The
// low-resolution samples that the adjoint at the tile's pixels reads, mirrored
// copies included, form a window [Ilo, Ihi] x [Jlo, Jhi] of the grid: a pixel
// i reads samples (i + R) / F - t (t < NS) or, within R of an edge, samples
// next to that same edge, which lie in the tile's own window for a mirrored
// boundary (a periodic one would reach the opposite edge).  The block stages
// the rows of x those samples cover, forms r = A x - y on the window in LDS
// with the additions of k_sr_forward (each row's taps first, then across
// rows), and takes the adjoint at its pixels from LDS as k_sr_adjoint_step
// does, so both forms give the same bits.
template <int TH, int TW>
struct XsGeo {
    static constexpr int BS = 9, F = 2, R = 4, NS = 5;
    // samples per window side: the tile's pixels reach ceil((n - 1) / F) + 1
    // distinct values of (i + R) / F, each with NS - 1 more below it
    static constexpr int NI = (TH - 1 + F - 1) / F + NS;
    static constexpr int NJ = (TW - 1 + F - 1) / F + NS;
    static constexpr int XR = F * (NI - 1) + BS;  // staged rows and columns of x
    static constexpr int XC = F * (NJ - 1) + BS;
};

template <int TH, int TW, int NT>
struct SRWindow {
    using G = XsGeo<TH, TW>;
    static constexpr int TILE_H = TH, TILE_W = TW, THREADS = NT;
    static constexpr int BS = G::BS, F = G::F, R = G::R, NS = G::NS;
    static constexpr int XN = G::XR * G::XC, HN = G::XR * G::NJ, RN = G::NI * G::NJ;  // LDS floats
    static constexpr int KX = (XN + NT - 1) / NT, KH = (HN + NT - 1) / NT, KR = (RN + NT - 1) / NT;
    int Ilo, Jlo, ni, nj, xr, xc, pr0, pc0;
    float xs[KX], yv[KR];

    // Issue the loads of the tile at (i0, j0): x over the window's rows and
    // columns and y over the window.  A tile outside the image loads nothing.
    __device__ __forceinline__ void load(const float* __restrict__ x, const float* __restrict__ y,
                                         const SRGeom& g, int i0, int j0, int tid) {
        const bool any = i0 < g.n1 && j0 < g.n2;
        const int imax = min(i0 + TH, g.n1) - 1, jmax = min(j0 + TW, g.n2) - 1;
        Ilo = max(0, (i0 + R) / F - (NS - 1));
        Jlo = max(0, (j0 + R) / F - (NS - 1));
        ni = any ? min(g.m1 - 1, (imax + R) / F) - Ilo + 1 : 0;
        nj = any ? min(g.m2 - 1, (jmax + R) / F) - Jlo + 1 : 0;
        xr = any ? F * (ni - 1) + BS : 0;
        xc = any ? F * (nj - 1) + BS : 0;
        pr0 = F * Ilo - R;  // padded position of the first staged row and column
        pc0 = F * Jlo - R;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int e = tid + k * NT, t = e / G::NJ, q = e % G::NJ;
            yv[k] = e < RN && t < ni && q < nj ? y[(size_t)(Ilo + t) * g.m2 + Jlo + q] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const int e = tid + k * NT, a = e / G::XC, b = e % G::XC;
            xs[k] = e < XN && a < xr && b < xc
                        ? x[(size_t)src_index<0>(pr0 + a, g.n1) * g.n2 + src_index<0>(pc0 + b, g.n2)]
                        : 0.f;
        }
    }

    // Form r on the window in Rw (X and H: LDS scratch); every thread of the
    // block calls it (three barriers).
    __device__ __forceinline__ void build(float* X, float* H, float* Rw, const Taps& taps, int tid) const {
#pragma unroll
        for (int k = 0; k < KX; ++k)
            if (tid + k * NT < XN) X[tid + k * NT] = xs[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            const int e = tid + k * NT, a = e / G::NJ, q = e % G::NJ;
            if (e < HN && a < xr && q < nj) {
                const float* row = X + a * G::XC + F * q;
                float ra = 0.f;
#pragma unroll
                for (int b = 0; b < BS; ++b) ra = fmaf(taps.t[b], row[b], ra);
                H[e] = ra;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int e = tid + k * NT, t = e / G::NJ, q = e % G::NJ;
            if (e < RN && t < ni && q < nj) {
                const float* col = H + F * t * G::NJ + q;
                float acc = 0.f;
#pragma unroll
                for (int a = 0; a < BS; ++a) acc = fmaf(taps.t[a], col[a * G::NJ], acc);
                Rw[e] = acc - yv[k];
            }
        }
        __syncthreads();
    }

    // (A^T r)(i, j) at a pixel of the tile, from the window in Rw.
    __device__ __forceinline__ float grad(const float* Rw, int i, int j, const SRGeom& g, const Taps& taps) const {
        const RLds rd{Rw, G::NJ, Ilo, Jlo};
        return i >= R && i < g.n1 - R && j >= R && j < g.n2 - R ? sr_adjoint_interior<BS, F>(rd, i, j, taps)
                                                                  : sr_adjoint_at<0, BS, F>(rd, i, j, g, taps);
    }
};

// Everything a kernel that finishes an iteration needs for the next
// iteration's x-step (9-tap, factor-2, mirrored operator), in device memory:
// it reads x (its own argument) and y, writes xo (not aliasing x) and z.
struct SRStepArgs {
    SRGeom g;
    Taps taps;
    StepScalars s;
    const float* y;
    float* xo;
    float* z;
};

// Rows per block of the kernels that finish an iteration with the next one's
// x-step (the single-image gather and the solver's epilogue split each 32-row
// tile over four blocks, one thread per pixel).
constexpr int kNextStepRows = 8;

// The next iteration's x-step for the block's tile after the dual update.
// Each thread holds one pixel (i, j) of the tile (valid: inside the image)
// with this iteration's x, v and u there; x_next goes to ns->xo and
// x_next + u to ns->z.  win holds the tile's window loads (issued at the
// start of the kernel); every thread of the block calls this (it builds the
// window in LDS).
template <class W>
__device__ __forceinline__ void next_xstep(const W& win, const SRStepArgs* __restrict__ ns, int i, int j,
                                           bool valid, float xv, float vv, float uv) {
    static_assert(W::TILE_H * W::TILE_W == W::THREADS, "one pixel per thread");
    __shared__ float X[W::XN];
    __shared__ float H[W::HN];
    __shared__ float Rw[W::RN];
    win.build(X, H, Rw, ns->taps, threadIdx.x);
    if (!valid) return;
    const SRGeom g = ns->g;
    const size_t idx = (size_t)i * g.n2 + j;
    const float xn = xstep_value(win.grad(Rw, i, j, g, ns->taps), xv, vv, uv, ns->s);
    ns->xo[idx] = xn;
    ns->z[idx] = xn + uv;
}

}  // namespace dsnlm
