// Linearized plug-and-play ADMM (Section 2, Algorithm 1) on gfx950.
//
// One iteration k:
//   x <- Pi_C(mu (alpha x + rho (v - u) - grad f(x)))        (linearized x-step)
//   z  = x + u                                               (denoiser input)
//   v <- W_k z, W_k = W(z) while k <= k0, else W_{k0}         (DSG-NLM)
//   u <- u + x - v                                           (dual update)
// with mu = 1/(alpha + rho), alpha = 1/gamma.  grad f is
//   super-resolution (Section 4.1): A^T (A x - y), A = decimation after a
//     separable blur with mirrored or periodic boundary;
//   single-photon imaging (Section 4.2): phi'(x_i) per pixel.
// The forward operator and its exact adjoint are evaluated directly (no FFT):
// the adjoint gathers, for each high-resolution pixel, every low-resolution
// sample whose blur footprint covers it or one of its mirrored/wrapped copies.
// Residual norms are reduced in two fixed-order stages (per-block partials,
// then one block), so repeated runs give identical bits.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "sr_step.h"

namespace dsnlm {

int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
int prepare_handle(int n1, int n2, int S, int P, float h, dsnlm_weights** out);
ImgDesc base_desc(const dsnlm_weights* w);

namespace {



// r = A x - y on the low-resolution grid (y may be null: r = A x).
// BS > 0 fixes the blur size and F the factor at compile time (the loops
// unroll, so all BS^2 loads of a sample are in flight together); BS = 0 takes
// both from g.  Both forms add in the same order.
template <int BOUNDARY, int BS, int F>
__global__ void __launch_bounds__(256)
k_sr_forward(const float* __restrict__ x, const float* __restrict__ y, float* __restrict__ r,
             SRGeom g, Taps taps) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= g.m1 * g.m2) return;
    const int I = idx / g.m2, J = idx - I * g.m2;
    float acc = 0.f;
    if constexpr (BS > 0) {
        constexpr int R = (BS - 1) / 2;
        int jj[BS];
#pragma unroll
        for (int b = 0; b < BS; ++b) jj[b] = src_index<BOUNDARY>(F * J + b - R, g.n2);
#pragma unroll
        for (int a = 0; a < BS; ++a) {
            const float* row = x + (size_t)src_index<BOUNDARY>(F * I + a - R, g.n1) * g.n2;
            float ra = 0.f;
#pragma unroll
            for (int b = 0; b < BS; ++b) ra = fmaf(taps.t[b], row[jj[b]], ra);
            acc = fmaf(taps.t[a], ra, acc);
        }
    } else {
        for (int a = 0; a < g.bs; ++a) {
            const int i = src_index<BOUNDARY>(g.f * I + a - g.R, g.n1);
            const float* row = x + (size_t)i * g.n2;
            float ra = 0.f;
            for (int b = 0; b < g.bs; ++b) {
                const int j = src_index<BOUNDARY>(g.f * J + b - g.R, g.n2);
                ra = fmaf(taps.t[b], row[j], ra);
            }
            acc = fmaf(taps.t[a], ra, acc);
        }
    }
    r[idx] = y ? acc - y[idx] : acc;
}


template <int BOUNDARY, int BS, int F>
__global__ void __launch_bounds__(256)
k_sr_adjoint_step(const float* __restrict__ r, float* __restrict__ x, const float* __restrict__ v,
                  const float* __restrict__ u, float* __restrict__ z, SRGeom g, Taps taps,
                  StepScalars s, int step) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= g.n1 * g.n2) return;
    const int i = idx / g.n2, j = idx - i * g.n2;
    const RGlobal rd{r, g.m2};
    float grad;
    if constexpr (BS > 0) {
        constexpr int R = (BS - 1) / 2;
        if (i >= R && i < g.n1 - R && j >= R && j < g.n2 - R)
            grad = sr_adjoint_interior<BS, F>(rd, i, j, taps);
        else
            grad = sr_adjoint_at<BOUNDARY, BS, F>(rd, i, j, g, taps);
    } else {
        grad = sr_adjoint_at<BOUNDARY, BS, F>(rd, i, j, g, taps);
    }
    if (!step) {
        x[idx] = grad;
        return;
    }
    xstep_store(grad, x, v, u, x, z, idx, s);
}

// The x-step of the 9-tap, factor-2 operator with mirrored boundary (the
// super-resolution setting of Section 4.1) in one launch: one block per
// kXsTH x kXsTW tile forms r = A x - y on the tile's window in LDS and takes
// the adjoint, clip and z = x + u from it (SRWindow).  x is read and xo
// written: they must not alias, since every block reads x beyond its own tile.
constexpr int kXsTH = 8, kXsTW = 64, kXsThreads = 512;

template <int TH, int TW>
__global__ void __launch_bounds__(kXsThreads)
k_sr_step_tile(const float* __restrict__ x, const float* __restrict__ y, float* __restrict__ xo,
               const float* __restrict__ v, const float* __restrict__ u, float* __restrict__ z, SRGeom g,
               Taps taps, StepScalars s) {
    using W = SRWindow<TH, TW, kXsThreads>;
    constexpr int NT = kXsThreads, KP = TH * TW / NT;
    static_assert(TH * TW % NT == 0, "whole pixels per thread");
    __shared__ float X[W::XN];
    __shared__ float H[W::HN];
    __shared__ float Rw[W::RN];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;
    // every global load is issued before the first wait: the pixels' x, v, u
    // and the window's x and y (their latency overlaps)
    float xv[KP], vv[KP], uv[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int e = tid + k * NT, i = i0 + e / TW, j = j0 + e % TW;
        const size_t idx = i < g.n1 && j < g.n2 ? (size_t)i * g.n2 + j : 0;
        xv[k] = x[idx];
        vv[k] = v[idx];
        uv[k] = u[idx];
    }
    W win;
    win.load(x, y, g, i0, j0, tid);
    win.build(X, H, Rw, taps, tid);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int e = tid + k * NT, i = i0 + e / TW, j = j0 + e % TW;
        if (i >= g.n1 || j >= g.n2) continue;
        const size_t idx = (size_t)i * g.n2 + j;
        const float xn = xstep_value(win.grad(Rw, i, j, g, taps), xv[k], vv[k], uv[k], s);
        xo[idx] = xn;
        z[idx] = xn + uv[k];
    }
}

// Launch the forward blur/decimation (r = A x - y) and the adjoint step on
// st, with the compile-time form for the 9-tap, factor-2 operator of Section
// 4.1 and the general form otherwise.
void launch_sr_forward(const SRGeom& g, const Taps& taps, int boundary, const float* x, const float* y,
                       float* r, hipStream_t st) {
    const dim3 grid((g.m1 * g.m2 + 255) / 256);
    const bool fixed = g.bs == 9 && g.f == 2;
    if (boundary == 0) {
        if (fixed) hipLaunchKernelGGL((k_sr_forward<0, 9, 2>), grid, dim3(256), 0, st, x, y, r, g, taps);
        else hipLaunchKernelGGL((k_sr_forward<0, 0, 0>), grid, dim3(256), 0, st, x, y, r, g, taps);
    } else {
        if (fixed) hipLaunchKernelGGL((k_sr_forward<1, 9, 2>), grid, dim3(256), 0, st, x, y, r, g, taps);
        else hipLaunchKernelGGL((k_sr_forward<1, 0, 0>), grid, dim3(256), 0, st, x, y, r, g, taps);
    }
}

void launch_sr_adjoint(const SRGeom& g, const Taps& taps, int boundary, const float* r, float* x,
                       const float* v, const float* u, float* z, const StepScalars& s, int step, hipStream_t st) {
    const dim3 grid((g.n1 * g.n2 + 255) / 256);
    const bool fixed = g.bs == 9 && g.f == 2;
    if (boundary == 0) {
        if (fixed) hipLaunchKernelGGL((k_sr_adjoint_step<0, 9, 2>), grid, dim3(256), 0, st, r, x, v, u, z, g, taps, s, step);
        else hipLaunchKernelGGL((k_sr_adjoint_step<0, 0, 0>), grid, dim3(256), 0, st, r, x, v, u, z, g, taps, s, step);
    } else {
        if (fixed) hipLaunchKernelGGL((k_sr_adjoint_step<1, 9, 2>), grid, dim3(256), 0, st, r, x, v, u, z, g, taps, s, step);
        else hipLaunchKernelGGL((k_sr_adjoint_step<1, 0, 0>), grid, dim3(256), 0, st, r, x, v, u, z, g, taps, s, step);
    }
}

// The operator takes the one-launch x-step (k_sr_step_tile).
bool sr_step_fusable(const ladmm_operator* op, const SRGeom& g) {
    return op->kind == LADMM_OP_SR && op->boundary == 0 && g.bs == 9 && g.f == 2;
}

void launch_sr_step_tile(const SRGeom& g, const Taps& taps, const float* x, const float* y, float* xo,
                         const float* v, const float* u, float* z, const StepScalars& s, hipStream_t st) {
    const dim3 grid((g.n2 + kXsTW - 1) / kXsTW, (g.n1 + kXsTH - 1) / kXsTH);
    hipLaunchKernelGGL((k_sr_step_tile<kXsTH, kXsTW>), grid, dim3(kXsThreads), 0, st, x, y, xo, v, u, z, g, taps, s);
}

struct SPIScalars {
    float eta_over_K;  // eta / K
    float K;
    float t_min;
};

__device__ __forceinline__ float spi_dphi(float t, float ones, const SPIScalars& q) {
    t = fmaxf(t, q.t_min);
    const float a = q.eta_over_K * t;
    const float e = expf(-a);
    const float denom = -expm1f(-a);  // 1 - exp(-eta t / K)
    return q.eta_over_K * ((q.K - ones) - ones * e / denom);
}

// SPI: x <- clip(mu (alpha x + rho (v - u) - phi'(x))); z = x + u
// (step == 0: write phi'(x) into z).
__global__ void __launch_bounds__(256)
k_spi_step(float* __restrict__ x, const float* __restrict__ v, const float* __restrict__ u,
           float* __restrict__ z, const unsigned char* __restrict__ ones, int n, SPIScalars q,
           StepScalars s, int step) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n) return;
    const float xv = x[idx];
    const float grad = spi_dphi(xv, (float)ones[idx], q);
    if (!step) {
        z[idx] = grad;
        return;
    }
    float xn = s.mu * (s.alpha * xv + s.rho * (v[idx] - u[idx]) - grad);
    xn = fminf(fmaxf(xn, s.lo), s.hi);
    x[idx] = xn;
    z[idx] = xn + u[idx];
}

// Threads of an epilogue block: one per pixel of its 8 x 64 rows.
constexpr int kEpilogueThreads = 512;

// v_new = z + B'/m (denoiser output); u <- u + x - v_new; v <- v_new; per-block
// partial sums of (x - v_new)^2 and (v_new - v_old)^2.  The blocks follow the
// single-image gather's geometry (a 32 x 64 tile's rows split over gridDim.z
// blocks), so both leave the same number of partials per iteration.
__global__ void __launch_bounds__(kEpilogueThreads)
k_ladmm_epilogue(const float* z, const float* __restrict__ bp, const unsigned long long* __restrict__ key,
                 const float* __restrict__ x, float* __restrict__ v, float* __restrict__ u, int n1, int n2,
                 float* __restrict__ partials, const SRStepArgs* __restrict__ ns) {
    constexpr int TH = 32, TW = 64;
    const float m = __uint_as_float((unsigned)(*key >> 32));
    const int rows = TH / (int)gridDim.z;
    const int i0 = (int)blockIdx.y * TH + (int)blockIdx.z * rows, j0 = (int)blockIdx.x * TW;
    // with ns set, the block ends with the next iteration's x-step for its
    // rows (kNextStepRows, one pixel per thread): its window loads go out first
    using W = SRWindow<kNextStepRows, TW, kEpilogueThreads>;
    W win;
    if (ns) win.load(x, ns->y, ns->g, i0, j0, threadIdx.x);
    float p = 0.f, d = 0.f;
    float kx = 0.f, kv = 0.f, ku = 0.f;  // this thread's pixel (the loop runs once when ns is set)
    bool kin = false;
    for (int e = threadIdx.x; e < rows * TW; e += kEpilogueThreads) {
        const int gi = i0 + e / TW, gj = j0 + e % TW;
        if (gi >= n1 || gj >= n2) continue;
        const size_t idx = (size_t)gi * n2 + gj;
        const float vn = z[idx] + bp[idx] / m;
        const float xv = x[idx];
        const float vo = v[idx];
        const float un = u[idx] + xv - vn;
        u[idx] = un;
        v[idx] = vn;
        p = fmaf(xv - vn, xv - vn, p);
        d = fmaf(vn - vo, vn - vo, d);
        kx = xv;
        kv = vn;
        ku = un;
        kin = true;
    }
    if (ns) {
        const int e = threadIdx.x;
        next_xstep(win, ns, i0 + e / TW, j0 + e % TW, kin, kx, kv, ku);
    }
    if (!partials) return;
    constexpr int NW = kEpilogueThreads / 64;
    static_assert(NW == 8, "the fixed-order block sum below adds eight wave sums");
    __shared__ float wsum[2][NW];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        p += __shfl_xor(p, off, 64);
        d += __shfl_xor(d, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        wsum[0][threadIdx.x >> 6] = p;
        wsum[1][threadIdx.x >> 6] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int b = ((int)blockIdx.z * (int)gridDim.y + (int)blockIdx.y) * (int)gridDim.x + (int)blockIdx.x;
#pragma unroll
        for (int c = 0; c < 2; ++c)
            partials[2 * b + c] = ((wsum[c][0] + wsum[c][1]) + (wsum[c][2] + wsum[c][3])) +
                                  ((wsum[c][4] + wsum[c][5]) + (wsum[c][6] + wsum[c][7]));
    }
}

// Iteration blockIdx.x: out[2k] = sqrt(sum_p / n), out[2k+1] = rho sqrt(sum_d / n)
// from its nblk partial pairs at partials + k * stride; fixed order.
__global__ void __launch_bounds__(256)
k_residual_final(const float* __restrict__ partials, size_t stride, int nblk, int n, float rho,
                 float* __restrict__ out) {
    const float* pk = partials + blockIdx.x * stride;
    __shared__ double sp[256], sd[256];
    double p = 0.0, d = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        p += pk[2 * b];
        d += pk[2 * b + 1];
    }
    sp[threadIdx.x] = p;
    sd[threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sp[threadIdx.x] += sp[threadIdx.x + w];
            sd[threadIdx.x] += sd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = (float)sqrt(sp[0] / n);
        out[2 * blockIdx.x + 1] = (float)(rho * sqrt(sd[0] / n));
    }
}

// ---- power iteration helpers -------------------------------------------
__device__ __forceinline__ float hash_uniform(unsigned k) {
    // integer hash (xorshift-multiply), mapped to [-1, 1)
    k ^= k >> 16;
    k *= 0x7feb352dU;
    k ^= k >> 15;
    k *= 0x846ca68bU;
    k ^= k >> 16;
    return (float)(k >> 8) * (2.0f / 16777216.0f) - 1.0f;
}

__global__ void k_fill_hash(float* __restrict__ v, int n) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < n) v[idx] = hash_uniform((unsigned)idx * 2654435761u + 12345u);
}

// partials[b] = (sum v.g, sum g.g) over block b
__global__ void __launch_bounds__(256)
k_dot2(const float* __restrict__ v, const float* __restrict__ g, int n, double* __restrict__ partials) {
    __shared__ double s0[256], s1[256];
    const int idx = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (idx < n) {
        a = (double)v[idx] * g[idx];
        b = (double)g[idx] * g[idx];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s0[0];
        partials[2 * blockIdx.x + 1] = s1[0];
    }
}

// out[0] = sum v.g (Rayleigh quotient, v unit), out[1] = ||g||
__global__ void __launch_bounds__(256)
k_dot2_final(const double* __restrict__ partials, int nblk, double* __restrict__ out) {
    __shared__ double s0[256], s1[256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) {
        a += partials[2 * k];
        b += partials[2 * k + 1];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = sqrt(s1[0]);
    }
}

__global__ void k_scale_into(const float* __restrict__ g, const double* __restrict__ nrm,
                             float* __restrict__ v, int n) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < n) v[idx] = (float)(g[idx] / nrm[1]);
}

__global__ void k_normalize(float* __restrict__ v, const double* __restrict__ nrm, int n) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < n) v[idx] = (float)(v[idx] / nrm[1]);
}

// ---- host helpers --------------------------------------------------------
inline int blocks(size_t n) { return (int)((n + 255) / 256); }

struct OpView {
    SRGeom g;
    Taps taps;
    SPIScalars q;
};

int check_operator(const ladmm_operator* op, bool need_y, const char* who, OpView* ov) {
    std::string w(who);
    if (!op) return fail(DSNLM_EINVAL, w + ": null operator");
    if (op->n1 < 1 || op->n2 < 1) return fail(DSNLM_EINVAL, w + ": image must be at least 1x1");
    if ((long long)op->n1 * op->n2 > (1LL << 31) - 1)
        return fail(DSNLM_EUNSUPPORTED, w + ": images above 2^31-1 pixels are not supported");
    std::memset(ov, 0, sizeof(*ov));
    if (op->kind == LADMM_OP_SR) {
        if (!op->taps) return fail(DSNLM_EINVAL, w + ": null blur taps");
        if (op->blur_size < 1 || op->blur_size > kMaxTaps || op->blur_size % 2 == 0)
            return fail(DSNLM_EINVAL, w + ": blur_size must be odd and <= 31");
        if (op->factor < 1 || op->factor > 8) return fail(DSNLM_EINVAL, w + ": factor must be in 1..8");
        if (op->boundary != 0 && op->boundary != 1) return fail(DSNLM_EINVAL, w + ": boundary must be 0 or 1");
        const int R = (op->blur_size - 1) / 2;
        if (R >= op->n1 || R >= op->n2)
            return fail(DSNLM_EINVAL, w + ": blur radius must be smaller than the image");
        for (int k = 0; k < op->blur_size; ++k)
            if (!std::isfinite(op->taps[k])) return fail(DSNLM_EINVAL, w + ": non-finite blur tap");
        if (need_y && !op->y) return fail(DSNLM_EINVAL, w + ": null observation y");
        ov->g = SRGeom{op->n1, op->n2, (op->n1 + op->factor - 1) / op->factor,
                       (op->n2 + op->factor - 1) / op->factor, op->factor, op->blur_size, R};
        for (int k = 0; k < op->blur_size; ++k) ov->taps.t[k] = op->taps[k];
        return DSNLM_OK;
    }
    if (op->kind == LADMM_OP_SPI) {
        if (!op->ones) return fail(DSNLM_EINVAL, w + ": null counts");
        if (op->K < 1 || op->K > 255) return fail(DSNLM_EINVAL, w + ": K must be in 1..255");
        if (!std::isfinite(op->eta) || !(op->eta > 0.f)) return fail(DSNLM_EINVAL, w + ": eta must be > 0");
        if (!std::isfinite(op->t_min) || !(op->t_min > 0.f)) return fail(DSNLM_EINVAL, w + ": t_min must be > 0");
        ov->q = SPIScalars{op->eta / (float)op->K, (float)op->K, op->t_min};
        return DSNLM_OK;
    }
    return fail(DSNLM_EINVAL, w + ": unknown operator kind");
}

int check_params(const ladmm_params* p, int n1, int n2, const char* who, float* h_eff) {
    std::string w(who);
    if (!p) return fail(DSNLM_EINVAL, w + ": null params");
    if (!(p->lambda > 0.f) || !(p->rho > 0.f) || !(p->gamma > 0.f) || !std::isfinite(p->lambda) ||
        !std::isfinite(p->rho) || !std::isfinite(p->gamma))
        return fail(DSNLM_EINVAL, w + ": lambda, rho and gamma must be finite and > 0");
    if (!(p->lo < p->hi) || !std::isfinite(p->lo) || !std::isfinite(p->hi))
        return fail(DSNLM_EINVAL, w + ": need finite lo < hi");
    if (p->freeze_after < 1) return fail(DSNLM_EINVAL, w + ": freeze_after must be >= 1");
    if (p->denoiser != 0 && p->denoiser != 1) return fail(DSNLM_EINVAL, w + ": denoiser must be 0 or 1");
    if (p->denoiser == 1 && !half_lds_fits(p->S, p->P, kNLM))
        return fail(DSNLM_EUNSUPPORTED, w + ": plain NLM for these S and P");
    if (p->iters < 0) return fail(DSNLM_EINVAL, w + ": iters must be >= 0");
    if (!std::isfinite(p->h)) return fail(DSNLM_EINVAL, w + ": h must be finite");
    const float h = p->h > 0.f ? p->h : std::sqrt(p->lambda / p->rho);
    *h_eff = h;
    return check_denoiser_args(n1, n2, p->S, p->P, h, who);
}

// Scratch carried by the weights handle for the solver (grow-only).
float* scratch_floats(dsnlm_weights* w, size_t n, int* rc) {
    if (w->scratch_cap < n) {
        if (w->scratch) (void)hipFree(w->scratch);
        w->scratch = nullptr;
        w->scratch_cap = 0;
        hipError_t e = hipMalloc(&w->scratch, n * sizeof(float));
        if (e != hipSuccess) {
            *rc = check_hip(e, "solver scratch");
            return nullptr;
        }
        w->scratch_cap = n;
    }
    *rc = DSNLM_OK;
    return w->scratch;
}

// Floats per iteration slot of the residual partials: two per gather (or
// epilogue) block, and at least one per 256 pixels (the CG solver's dot
// products use slot 0).
size_t partial_stride(int n1, int n2) {
    const size_t a = 2 * (size_t)gather_blocks(n1, n2), b = (size_t)blocks((size_t)n1 * n2);
    return ((a > b ? a : b) + 63) & ~(size_t)63;
}

// The denoising and dual halves of an iteration (shared by Algorithm 1 and
// the standard ADMM comparator): v = D(z) with z = x + u already in w->zbuf,
// u <- u + x - v, and checkpoints.  With want_res the iteration's residual
// partials go to `partials` (gather_blocks pairs, reduced by the caller).
// A frozen iteration on the half-window path does the dual half inside the
// apply's gather (m is known), so no separate update kernel runs.
int enqueue_denoise_dual(const ladmm_params* p, int k, dsnlm_weights* w, float* x, float* v, float* u,
                         float* partials, bool want_res, float* ckpt, hipStream_t st,
                         const SRStepArgs* ns = nullptr) {
    const int n = w->n1 * w->n2;
    float* z = w->zbuf;
    ImgDesc d = base_desc(w);
    d.x = z;
    int rc;
    bool fused = false;
    if (p->denoiser == 1) {
        // plain NLM of z guided by z: writes its increment into B' and m = 1
        rc = check_hip(hipMemcpyAsync(w->guide, z, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st),
                       "copy guide");
        d.z = w->guide;
        d.y = nullptr;
        if (!rc) rc = check_hip(launch_half(kNLM, p->S, p->P, d, nullptr, nullptr, 0, st), "plain NLM");
    } else if (k <= p->freeze_after) {
        // adaptive weights: guide = the denoiser's own input z.  On the half
        // window only pass A's pad reads it (into the mirrored copy that the
        // later sweeps and frozen applies use), so a solve's own handle takes z
        // as it is; otherwise the handle keeps a copy (the full-window sweeps
        // read the guide itself, and a caller's handle may be differentiated)
        d.z = z;
        const bool direct = w->solver_owned && sweep_takes_half(kPassA, p->S, p->P, d) &&
                            sweep_takes_half(kPassBApply, p->S, p->P, d) && sweep_takes_half(kApply, p->S, p->P, d);
        rc = DSNLM_OK;
        if (!direct) {
            rc = check_hip(hipMemcpyAsync(w->guide, z, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st),
                           "copy guide");
            d.z = w->guide;
        }
        if (!rc) rc = check_hip(launch_sweep(kPassA, p->S, p->P, d, nullptr, nullptr, 0, st), "pass A");
        if (!rc) rc = check_hip(launch_sweep(kPassBApply, p->S, p->P, d, nullptr, nullptr, 0, st), "pass B");
    } else {
        fused = sweep_takes_half(kApply, p->S, p->P, d);
        if (fused) {
            d.lx = x;
            d.lv = v;
            d.lu = u;
            d.lres = want_res ? partials : nullptr;
            d.lstep = ns;
        }
        rc = check_hip(launch_sweep(kApply, p->S, p->P, d, nullptr, nullptr, 0, st), "apply sweep");
    }
    if (rc) return rc;
    if (!fused) {
        ProfScope prof(DSNLM_K_LADMM, st);
        const dim3 grid((w->n2 + 63) / 64, (w->n1 + 31) / 32, kGatherSplit);
        hipLaunchKernelGGL(k_ladmm_epilogue, grid, dim3(kEpilogueThreads), 0, st, z, w->bp, w->key, x, v, u, w->n1, w->n2,
                           want_res ? partials : nullptr, ns);
        rc = check_hip(hipGetLastError(), "dual update");
        if (rc) return rc;
    }
    w->applied = true;
    if (ckpt) {
        const size_t b = (size_t)n * sizeof(float);
        rc = check_hip(hipMemcpyAsync(ckpt, x, b, hipMemcpyDeviceToDevice, st), "checkpoint");
        if (!rc) rc = check_hip(hipMemcpyAsync(ckpt + n, v, b, hipMemcpyDeviceToDevice, st), "checkpoint");
        if (!rc) rc = check_hip(hipMemcpyAsync(ckpt + 2 * (size_t)n, u, b, hipMemcpyDeviceToDevice, st), "checkpoint");
        if (!rc) rc = check_hip(hipMemcpyAsync(ckpt + 3 * (size_t)n, z, b, hipMemcpyDeviceToDevice, st), "checkpoint");
    }
    return rc;
}

// Reduce the residual partials of `iters` consecutive slots into res
// ([iters][2]).
int enqueue_residuals(const float* partials, int n1, int n2, int iters, float rho, float* res, hipStream_t st) {
    ProfScope prof(DSNLM_K_LADMM, st);
    hipLaunchKernelGGL(k_residual_final, dim3(iters), dim3(256), 0, st, partials, partial_stride(n1, n2),
                       gather_blocks(n1, n2), n1 * n2, rho, res);
    return check_hip(hipGetLastError(), "residual reduction");
}

// Enqueue iteration k of Algorithm 1.  The x-step reads x and writes xo: the
// same buffer (in place, two launches for the super-resolution operator) or,
// for an operator with sr_step_fusable, another one (one launch).  The rest of
// the iteration works on xo.  With stepped set the previous iteration's last
// kernel has already taken this x-step; with ns set this iteration's last
// kernel takes the next one (ns: device arguments, reading xo).  lr: scratch
// for the low-resolution residual (SR); partials: this iteration's slot of
// residual partials (written when want_res); ckpt: device [4][n] or null.
int enqueue_step(const ladmm_operator* op, const OpView& ov, const ladmm_params* p, float h, int k,
                 dsnlm_weights* w, const float* x, float* xo, float* v, float* u, float* lr, float* partials,
                 bool want_res, float* ckpt, hipStream_t st, bool stepped = false, const SRStepArgs* ns = nullptr) {
    (void)h;
    const int n = op->n1 * op->n2;
    const float alpha = 1.0f / p->gamma;
    StepScalars s{alpha, p->rho, 1.0f / (alpha + p->rho), p->lo, p->hi};
    float* z = w->zbuf;
    if (xo != x && !sr_step_fusable(op, ov.g)) return fail(DSNLM_EINVAL, "x-step: out of place for this operator");
    if (!stepped) {
        ProfScope prof(DSNLM_K_LADMM, st);
        if (xo != x) {
            launch_sr_step_tile(ov.g, ov.taps, x, op->y, xo, v, u, z, s, st);
        } else if (op->kind == LADMM_OP_SR) {
            launch_sr_forward(ov.g, ov.taps, op->boundary, x, op->y, lr, st);
            launch_sr_adjoint(ov.g, ov.taps, op->boundary, lr, xo, v, u, z, s, 1, st);
        } else {
            hipLaunchKernelGGL(k_spi_step, dim3(blocks(n)), dim3(256), 0, st, xo, v, u, z, op->ones, n, ov.q, s, 1);
        }
        int rc = check_hip(hipGetLastError(), "x-step");
        if (rc) return rc;
    }
    return enqueue_denoise_dual(p, k, w, xo, v, u, partials, want_res, ckpt, st, ns);
}

// ---- standard plug-and-play ADMM with a conjugate-gradient inversion (the
// comparator of Fig. 2).  The x-update solves (A^T A + rho I) x = A^T y +
// rho (v - u); CG scalars live on the device (no host round trip).

struct CGScalars {
    float rr, pq, alpha, beta;
};

// fixed-order block partial of a dot product
__device__ __forceinline__ void block_partial(float val, float* partials) {
    __shared__ float sh[256];
    sh[threadIdx.x] = val;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// r = A^T y + rho (v - u) - (A^T A x + rho x) (Mx holds A^T A x); p = r
__global__ void __launch_bounds__(256)
k_cg_start(const float* __restrict__ aty, const float* __restrict__ Mx, const float* __restrict__ x,
           const float* __restrict__ v, const float* __restrict__ u, float* __restrict__ r, float* __restrict__ pd,
           float rho, int n, float* __restrict__ partials) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    float val = 0.f;
    if (idx < n) {
        const float ri = aty[idx] + rho * (v[idx] - u[idx]) - (Mx[idx] + rho * x[idx]);
        r[idx] = ri;
        pd[idx] = ri;
        val = ri * ri;
    }
    block_partial(val, partials);
}

// q <- q + rho p (q held A^T A p); partial of p . q
__global__ void __launch_bounds__(256)
k_cg_pq(const float* __restrict__ pd, float* __restrict__ q, float rho, int n, float* __restrict__ partials) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    float val = 0.f;
    if (idx < n) {
        const float qi = q[idx] + rho * pd[idx];
        q[idx] = qi;
        val = pd[idx] * qi;
    }
    block_partial(val, partials);
}

// x += alpha p, r -= alpha q; partial of r . r
__global__ void __launch_bounds__(256)
k_cg_update(float* __restrict__ x, float* __restrict__ r, const float* __restrict__ pd, const float* __restrict__ q,
            const CGScalars* __restrict__ sc, int n, float* __restrict__ partials) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const float a = sc->alpha;
    float val = 0.f;
    if (idx < n) {
        x[idx] += a * pd[idx];
        const float ri = r[idx] - a * q[idx];
        r[idx] = ri;
        val = ri * ri;
    }
    block_partial(val, partials);
}

// p = r + beta p
__global__ void __launch_bounds__(256)
k_cg_dir(const float* __restrict__ r, float* __restrict__ pd, const CGScalars* __restrict__ sc, int n) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < n) pd[idx] = r[idx] + sc->beta * pd[idx];
}

// which: 0 -> rr, 1 -> pq and alpha = rr / pq, 2 -> beta = rr_new / rr, rr = rr_new
__global__ void __launch_bounds__(256) k_cg_reduce(const float* __restrict__ partials, int nblk, CGScalars* sc,
                                                   int which) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += partials[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const float t = (float)sh[0];
    if (which == 0) {
        sc->rr = t;
    } else if (which == 1) {
        sc->pq = t;
        sc->alpha = t > 0.f ? sc->rr / t : 0.f;
    } else {
        sc->beta = sc->rr > 0.f ? t / sc->rr : 0.f;
        sc->rr = t;
    }
}

__global__ void __launch_bounds__(256)
k_add(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ out, int n) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < n) out[idx] = a[idx] + b[idx];
}

// out = A^T A x (the low-resolution scratch lr holds A x)
void enqueue_AtA(const ladmm_operator* op, const OpView& ov, const float* x, float* lr, float* out,
                 hipStream_t st) {
    const int n = op->n1 * op->n2, mlr = ov.g.m1 * ov.g.m2;
    StepScalars s{};
    launch_sr_forward(ov.g, ov.taps, op->boundary, x, nullptr, lr, st);
    launch_sr_adjoint(ov.g, ov.taps, op->boundary, lr, out, nullptr, nullptr, nullptr, s, 0, st);
}

// Solver scratch layout inside the handle: [z: n][lr: m][xt: n][partials:
// slots x partial_stride] (one slot of residual partials per iteration of a
// solve; lr and xt for the super-resolution operator only, xt being the
// second x buffer of the one-launch x-step).
int ensure_solver_scratch(dsnlm_weights* w, const OpView& ov, const ladmm_operator* op, int slots, float** lr,
                          float** partials, float** xt = nullptr) {
    const size_t n = (size_t)op->n1 * op->n2;
    const bool sr = op->kind == LADMM_OP_SR;
    const size_t mlr = sr ? (size_t)ov.g.m1 * ov.g.m2 : 0;
    const size_t lead = (n + mlr + (sr ? n : 0) + 63) & ~(size_t)63;
    const size_t need = lead + (size_t)(slots < 1 ? 1 : slots) * partial_stride(op->n1, op->n2) + 64;
    int rc;
    float* base = scratch_floats(w, need, &rc);
    if (!base) return rc;
    w->zbuf = base;
    *lr = base + n;
    *partials = base + lead;
    if (xt) *xt = sr ? base + n + mlr : nullptr;
    return DSNLM_OK;
}

// ---- ladmm_solve's cache.  A solve is captured once into a HIP graph (all
// iterations, the adaptive ones included) for each distinct set of arguments
// (operator, parameters, state and output buffers, device) and replayed by
// later calls with the same arguments.  The graph runs on a library stream of
// the device, joined to the caller's stream by events; each entry owns its
// weights handle and solver scratch.

// Every iteration of a solve on stream st (ckpt/res: per-iteration slices).
int enqueue_solve(const ladmm_operator* op, const OpView& ov, const ladmm_params* p, float h, dsnlm_weights* w,
                  float* x, float* v, float* u, float* residuals, float* checkpoints, hipStream_t st,
                  const SRStepArgs* chain = nullptr) {
    float *lr, *partials, *xt;
    int rc = ensure_solver_scratch(w, ov, op, residuals ? p->iters : 1, &lr, &partials, &xt);
    const size_t n = (size_t)op->n1 * op->n2;
    const size_t stride = partial_stride(op->n1, op->n2);
    // With the one-launch x-step, x alternates between the state buffer and
    // xt; an odd count takes its first step in place, so the last lands in x.
    // With chain (device arguments: [0] writes xt, [1] writes x) and no
    // checkpoints (which keep each iteration's z), every iteration but the
    // last ends with the next one's x-step.
    const bool alt = sr_step_fusable(op, ov.g);
    const bool fold = alt && chain && !checkpoints;
    float* cur = x;
    bool stepped = false;
    for (int k = 1; k <= p->iters && !rc; ++k) {
        float* next = cur;
        if (alt && (k > 1 || p->iters % 2 == 0)) next = cur == x ? xt : x;
        const SRStepArgs* ns = fold && k < p->iters ? chain + (next == x ? 0 : 1) : nullptr;
        rc = enqueue_step(op, ov, p, h, k, w, cur, next, v, u, lr, partials + (residuals ? (k - 1) * stride : 0),
                          residuals != nullptr, checkpoints ? checkpoints + 4 * n * (size_t)(k - 1) : nullptr, st,
                          stepped, ns);
        stepped = ns != nullptr;
        cur = next;
    }
    // every iteration's residual norms in one fixed-order reduction at the end
    if (!rc && residuals) rc = enqueue_residuals(partials, op->n1, op->n2, p->iters, p->rho, residuals, st);
    return rc;
}

struct SolveKey {
    int device;
    ladmm_operator op;  // sizes and scalars only: the pointers are left null
    Taps taps;
    ladmm_params p;
    int want_res, want_ckpt;
};

// The graph of an entry reads and writes the entry's own copies of the state,
// the observation and the outputs, so one entry serves every call with the
// same sizes and parameters; the caller's buffers are copied in before and
// out after each replay (plain stream copies outside the graph).
struct SolveEntry {
    SolveKey key;
    dsnlm_weights* w = nullptr;
    float* buf = nullptr;          // x, v, u | observation y or counts | residuals | checkpoints
    float *x, *v, *u, *res, *ckpt;
    const float* y;
    const SRStepArgs* chain = nullptr;  // device [2]: the folded x-steps' arguments (or null)
    const unsigned char* ones;
    hipGraphExec_t exec = nullptr;  // null: the solve is enqueued step by step
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    unsigned long long used = 0;
};

constexpr int kSolveCacheSize = 4;
constexpr int kSolveDevices = 64;

struct SolveCache {
    std::mutex mu;
    std::vector<SolveEntry*> entries;
    hipStream_t stream[kSolveDevices] = {};
    unsigned long long tick = 0;
};
SolveCache g_solves;

void drop_entry(SolveEntry* e) {
    (void)hipStreamSynchronize(g_solves.stream[e->key.device]);
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->ev_in) (void)hipEventDestroy(e->ev_in);
    if (e->ev_out) (void)hipEventDestroy(e->ev_out);
    (void)hipFree(e->buf);
    dsnlm_weights_destroy(e->w);
    delete e;
}

// Find or create the entry of `key` (caller holds g_solves.mu); a new entry
// gets its handle, scratch and, when capture succeeds, its graph.
int solve_entry(const SolveKey& key, const ladmm_operator* op, const OpView& ov, float h, SolveEntry** out) {
    const int dev = key.device;
    if (dev < 0 || dev >= kSolveDevices) return fail(DSNLM_EUNSUPPORTED, "ladmm_solve: device index too large");
    for (SolveEntry* e : g_solves.entries)
        if (std::memcmp(&e->key, &key, sizeof(key)) == 0) {
            e->used = ++g_solves.tick;
            *out = e;
            return DSNLM_OK;
        }
    int rc;
    if (!g_solves.stream[dev]) {
        rc = check_hip(hipStreamCreateWithFlags(&g_solves.stream[dev], hipStreamNonBlocking), "ladmm_solve: stream");
        if (rc) return rc;
    }
    if ((int)g_solves.entries.size() >= kSolveCacheSize) {
        auto lru = g_solves.entries.begin();
        for (auto it = g_solves.entries.begin(); it != g_solves.entries.end(); ++it)
            if ((*it)->used < (*lru)->used) lru = it;
        drop_entry(*lru);
        g_solves.entries.erase(lru);
    }
    SolveEntry* e = new (std::nothrow) SolveEntry{};
    if (!e) return fail(DSNLM_ENOMEM, "ladmm_solve: host allocation failed");
    e->key = key;
    const ladmm_params* p = &key.p;
    const size_t n = (size_t)op->n1 * op->n2;
    const size_t nobs = op->kind == LADMM_OP_SR ? (size_t)ov.g.m1 * ov.g.m2 : (n + 3) / 4;  // floats
    const size_t nres = key.want_res ? 2 * (size_t)p->iters : 0;
    const size_t nck = key.want_ckpt ? 4 * n * (size_t)p->iters : 0;
    const size_t nargs = (2 * sizeof(SRStepArgs) + sizeof(float) - 1) / sizeof(float);
    const size_t r64 = 64;
    auto up = [&](size_t f) { return (f + r64 - 1) / r64 * r64; };
    rc = check_hip(hipMalloc(&e->buf, (3 * up(n) + up(nobs) + up(nres) + up(nck) + up(nargs)) * sizeof(float)),
                   "ladmm_solve: state buffers");
    if (rc) {
        delete e;
        return rc;
    }
    e->x = e->buf;
    e->v = e->x + up(n);
    e->u = e->v + up(n);
    float* obs = e->u + up(n);
    e->y = op->kind == LADMM_OP_SR ? obs : nullptr;
    e->ones = op->kind == LADMM_OP_SPI ? reinterpret_cast<const unsigned char*>(obs) : nullptr;
    e->res = key.want_res ? obs + up(nobs) : nullptr;
    e->ckpt = key.want_ckpt ? obs + up(nobs) + up(nres) : nullptr;
    ladmm_operator iop = *op;  // the operator as the graph sees it
    iop.y = e->y;
    iop.ones = e->ones;
    rc = prepare_handle(op->n1, op->n2, p->S, p->P, h, &e->w);
    if (!rc) e->w->solver_owned = true;
    float *lr, *partials, *xt;
    if (!rc) rc = ensure_solver_scratch(e->w, ov, op, key.want_res ? p->iters : 1, &lr, &partials, &xt);
    if (!rc && sr_step_fusable(op, ov.g)) {
        // the arguments of the x-steps folded into the iterations' last kernels
        const float alpha = 1.0f / p->gamma;
        SRStepArgs a[2];
        std::memset(a, 0, sizeof(a));
        for (int t = 0; t < 2; ++t) {
            a[t].g = ov.g;
            a[t].taps = ov.taps;
            a[t].s = StepScalars{alpha, p->rho, 1.0f / (alpha + p->rho), p->lo, p->hi};
            a[t].y = e->y;
            a[t].xo = t == 0 ? xt : e->x;
            a[t].z = e->w->zbuf;
        }
        SRStepArgs* dev = reinterpret_cast<SRStepArgs*>(obs + up(nobs) + up(nres) + up(nck));
        rc = check_hip(hipMemcpy(dev, a, sizeof(a), hipMemcpyHostToDevice), "ladmm_solve: step arguments");
        if (!rc) e->chain = dev;
    }
    if (!rc) rc = check_hip(prepare_sweeps(p->S, p->P), "sweep attributes");
    if (!rc) rc = check_hip(hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming), "ladmm_solve: event");
    if (!rc) rc = check_hip(hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming), "ladmm_solve: event");
    if (rc) {
        drop_entry(e);
        return rc;
    }
    hipStream_t is = g_solves.stream[dev];
    if (hipStreamBeginCapture(is, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        rc = enqueue_solve(&iop, ov, p, h, e->w, e->x, e->v, e->u, e->res, e->ckpt, is, e->chain);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(is, &graph);
        if (!rc && ec == hipSuccess && graph &&
            hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0) != hipSuccess)
            e->exec = nullptr;
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) {
            drop_entry(e);
            return rc;
        }
    }
    (void)hipGetLastError();  // a failed capture leaves the step-by-step path
    e->used = ++g_solves.tick;
    g_solves.entries.push_back(e);
    *out = e;
    return DSNLM_OK;
}

}  // namespace

// out = A^T A x for the super-resolution operator (lr: low-resolution scratch).
int sr_apply_AtA(const ladmm_operator* op, const float* x, float* lr, float* out, hipStream_t st) {
    OpView ov;
    int rc = check_operator(op, false, "sr_apply_AtA", &ov);
    if (rc) return rc;
    StepScalars s{};
    launch_sr_forward(ov.g, ov.taps, op->boundary, x, nullptr, lr, st);
    launch_sr_adjoint(ov.g, ov.taps, op->boundary, lr, out, nullptr, nullptr, nullptr, s, 0, st);
    return check_hip(hipGetLastError(), "A^T A");
}

}  // namespace dsnlm

using namespace dsnlm;

extern "C" {

int ladmm_step(const ladmm_operator* op, const ladmm_params* p, int k, dsnlm_weights** w, float* x, float* v,
               float* u, void* stream) {
    OpView ov;
    int rc = check_operator(op, true, "ladmm_step", &ov);
    if (rc) return rc;
    float h;
    rc = check_params(p, op->n1, op->n2, "ladmm_step", &h);
    if (rc) return rc;
    if (!w || !x || !v || !u) return fail(DSNLM_EINVAL, "ladmm_step: null pointer");
    if (k < 1) return fail(DSNLM_EINVAL, "ladmm_step: k is 1-based");
    const bool adaptive = k <= p->freeze_after || p->denoiser == 1;
    if (!adaptive && !*w)
        return fail(DSNLM_EINVAL, "ladmm_step: frozen iteration without built weights");
    if (*w && ((*w)->n1 != op->n1 || (*w)->n2 != op->n2))
        return fail(DSNLM_EINVAL, "ladmm_step: weights built for another image size");
    // frozen iterations reuse the handle's buffers, sized for its S and P
    if (!adaptive && ((*w)->S != p->S || (*w)->P != p->P))
        return fail(DSNLM_EINVAL, "ladmm_step: frozen iteration with S or P other than the weights'");
    if (adaptive) {
        rc = prepare_handle(op->n1, op->n2, p->S, p->P, h, w);
        if (rc) return rc;
    }
    float *lr, *partials;
    rc = ensure_solver_scratch(*w, ov, op, 1, &lr, &partials);
    if (rc) return rc;
    return enqueue_step(op, ov, p, h, k, *w, x, x, v, u, lr, partials, false, nullptr,
                        static_cast<hipStream_t>(stream));
}

int ladmm_solve(const ladmm_operator* op, const ladmm_params* p, float* x, float* v, float* u, float* residuals,
                float* checkpoints, void* stream) {
    OpView ov;
    int rc = check_operator(op, true, "ladmm_solve", &ov);
    if (rc) return rc;
    float h;
    rc = check_params(p, op->n1, op->n2, "ladmm_solve", &h);
    if (rc) return rc;
    if (!x || !v || !u) return fail(DSNLM_EINVAL, "ladmm_solve: null pointer");
    if (p->iters == 0) return DSNLM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (st) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        rc = check_hip(hipStreamIsCapturing(st, &cs), "ladmm_solve: capture status");
        if (rc) return rc;
        if (cs != hipStreamCaptureStatusNone)
            return fail(DSNLM_EINVAL, "ladmm_solve: the stream is being captured (the solve captures its own graph)");
    }
    int dev = 0;
    rc = check_hip(hipGetDevice(&dev), "ladmm_solve: hipGetDevice");
    if (rc) return rc;
    SolveKey key;
    std::memset(&key, 0, sizeof(key));
    key.device = dev;
    // field by field, so that the caller's struct padding never enters the key
    key.op.kind = op->kind;
    key.op.n1 = op->n1;
    key.op.n2 = op->n2;
    key.op.blur_size = op->blur_size;
    key.op.factor = op->factor;
    key.op.boundary = op->boundary;
    key.op.K = op->K;
    key.op.eta = op->eta;
    key.op.t_min = op->t_min;
    key.taps = ov.taps;  // the taps by value (the pointer is the caller's host array)
    key.p = *p;
    key.want_res = residuals != nullptr;
    key.want_ckpt = checkpoints != nullptr;
    std::lock_guard<std::mutex> lk(g_solves.mu);
    SolveEntry* e = nullptr;
    rc = solve_entry(key, op, ov, h, &e);
    if (rc) return rc;
    hipStream_t is = g_solves.stream[dev];
    // the internal stream runs after the caller's prior work, and the
    // caller's later work after the solve
    rc = check_hip(hipEventRecord(e->ev_in, st), "ladmm_solve: record");
    if (!rc) rc = check_hip(hipStreamWaitEvent(is, e->ev_in, 0), "ladmm_solve: wait");
    const size_t n = (size_t)op->n1 * op->n2, nb = n * sizeof(float);
    auto copy = [&](void* dst, const void* src, size_t bytes) {
        if (!rc) rc = check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, is), "ladmm_solve: copy");
    };
    copy(e->x, x, nb);
    copy(e->v, v, nb);
    copy(e->u, u, nb);
    if (op->kind == LADMM_OP_SR)
        copy(const_cast<float*>(e->y), op->y, (size_t)ov.g.m1 * ov.g.m2 * sizeof(float));
    else
        copy(const_cast<unsigned char*>(e->ones), op->ones, n);
    if (!rc) {
        if (e->exec) {
            rc = check_hip(hipGraphLaunch(e->exec, is), "ladmm_solve: graph launch");
        } else {
            ladmm_operator iop = *op;
            iop.y = e->y;
            iop.ones = e->ones;
            rc = enqueue_solve(&iop, ov, p, h, e->w, e->x, e->v, e->u, e->res, e->ckpt, is, e->chain);
        }
    }
    copy(x, e->x, nb);
    copy(v, e->v, nb);
    copy(u, e->u, nb);
    if (residuals) copy(residuals, e->res, 2 * (size_t)p->iters * sizeof(float));
    if (checkpoints) copy(checkpoints, e->ckpt, 4 * nb * (size_t)p->iters);
    if (!rc) rc = check_hip(hipEventRecord(e->ev_out, is), "ladmm_solve: record");
    if (!rc) rc = check_hip(hipStreamWaitEvent(st, e->ev_out, 0), "ladmm_solve: wait");
    if (rc) return rc;
    if (residuals) {
        // the documented synchronisation: residuals are checked on the host
        std::vector<float> host(2 * (size_t)p->iters);
        rc = check_hip(hipMemcpyAsync(host.data(), residuals, host.size() * sizeof(float), hipMemcpyDeviceToHost, st),
                       "copy residuals");
        if (!rc) rc = check_hip(hipStreamSynchronize(st), "ladmm_solve: synchronise");
        if (rc) return rc;
        for (float r : host)
            if (!std::isfinite(r)) return fail(DSNLM_ENONFINITE, "ladmm_solve: non-finite residual");
    }
    return DSNLM_OK;
}

int ladmm_apply_forward(const ladmm_operator* op, const float* x, float* out, void* stream) {
    OpView ov;
    int rc = check_operator(op, false, "ladmm_apply_forward", &ov);
    if (rc) return rc;
    if (op->kind != LADMM_OP_SR) return fail(DSNLM_EINVAL, "ladmm_apply_forward: super-resolution only");
    if (!x || !out) return fail(DSNLM_EINVAL, "ladmm_apply_forward: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ProfScope prof(DSNLM_K_LADMM, st);
    const int mlr = ov.g.m1 * ov.g.m2;
    launch_sr_forward(ov.g, ov.taps, op->boundary, x, nullptr, out, st);
    return check_hip(hipGetLastError(), "ladmm_apply_forward");
}

int ladmm_gradient(const ladmm_operator* op, const float* x, float* g, void* stream) {
    OpView ov;
    int rc = check_operator(op, true, "ladmm_gradient", &ov);
    if (rc) return rc;
    if (!x || !g) return fail(DSNLM_EINVAL, "ladmm_gradient: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = op->n1 * op->n2;
    StepScalars s{};
    if (op->kind == LADMM_OP_SPI) {
        ProfScope prof(DSNLM_K_LADMM, st);
        hipLaunchKernelGGL(k_spi_step, dim3(blocks(n)), dim3(256), 0, st, const_cast<float*>(x), nullptr, nullptr,
                           g, op->ones, n, ov.q, s, 0);
        return check_hip(hipGetLastError(), "ladmm_gradient");
    }
    float* lr = nullptr;
    rc = check_hip(hipMalloc(&lr, (size_t)ov.g.m1 * ov.g.m2 * sizeof(float)), "gradient scratch");
    if (rc) return rc;
    {
        ProfScope prof(DSNLM_K_LADMM, st);
        const int mlr = ov.g.m1 * ov.g.m2;
        launch_sr_forward(ov.g, ov.taps, op->boundary, x, op->y, lr, st);
        launch_sr_adjoint(ov.g, ov.taps, op->boundary, lr, g, nullptr, nullptr, nullptr, s, 0, st);
        rc = check_hip(hipGetLastError(), "ladmm_gradient");
    }
    hipError_t e = hipStreamSynchronize(st);
    (void)hipFree(lr);
    if (!rc) rc = check_hip(e, "gradient synchronise");
    return rc;
}

int ladmm_operator_norm2(const ladmm_operator* op, int iters, float* out, void* stream) {
    OpView ov;
    int rc = check_operator(op, false, "ladmm_operator_norm2", &ov);
    if (rc) return rc;
    if (op->kind != LADMM_OP_SR) return fail(DSNLM_EINVAL, "ladmm_operator_norm2: super-resolution only");
    if (!out || iters < 1) return fail(DSNLM_EINVAL, "ladmm_operator_norm2: need out and iters >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = op->n1 * op->n2;
    const int mlr = ov.g.m1 * ov.g.m2;
    float *v = nullptr, *g = nullptr, *lr = nullptr;
    double *part = nullptr, *red = nullptr;
    rc = check_hip(hipMalloc(&v, (size_t)n * sizeof(float)), "norm scratch");
    if (!rc) rc = check_hip(hipMalloc(&g, (size_t)n * sizeof(float)), "norm scratch");
    if (!rc) rc = check_hip(hipMalloc(&lr, (size_t)mlr * sizeof(float)), "norm scratch");
    if (!rc) rc = check_hip(hipMalloc(&part, 2 * (size_t)blocks(n) * sizeof(double)), "norm scratch");
    if (!rc) rc = check_hip(hipMalloc(&red, 2 * sizeof(double)), "norm scratch");
    StepScalars s{};
    if (!rc) {
        ProfScope prof(DSNLM_K_LADMM, st);
        hipLaunchKernelGGL(k_fill_hash, dim3(blocks(n)), dim3(256), 0, st, v, n);
        // normalise the start vector: reuse dot2 with g = v
        hipLaunchKernelGGL(k_dot2, dim3(blocks(n)), dim3(256), 0, st, v, v, n, part);
        hipLaunchKernelGGL(k_dot2_final, dim3(1), dim3(256), 0, st, part, blocks(n), red);
        hipLaunchKernelGGL(k_normalize, dim3(blocks(n)), dim3(256), 0, st, v, red, n);
        for (int it = 0; it < iters; ++it) {
            launch_sr_forward(ov.g, ov.taps, op->boundary, v, nullptr, lr, st);
            launch_sr_adjoint(ov.g, ov.taps, op->boundary, lr, g, nullptr, nullptr, nullptr, s, 0, st);
            hipLaunchKernelGGL(k_dot2, dim3(blocks(n)), dim3(256), 0, st, v, g, n, part);
            hipLaunchKernelGGL(k_dot2_final, dim3(1), dim3(256), 0, st, part, blocks(n), red);
            hipLaunchKernelGGL(k_scale_into, dim3(blocks(n)), dim3(256), 0, st, g, red, v, n);
        }
        rc = check_hip(hipGetLastError(), "power iteration");
    }
    double host[2] = {0, 0};
    if (!rc) rc = check_hip(hipMemcpyAsync(host, red, sizeof(host), hipMemcpyDeviceToHost, st), "copy norm");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "synchronise");
    (void)hipFree(v);
    (void)hipFree(g);
    (void)hipFree(lr);
    (void)hipFree(part);
    (void)hipFree(red);
    if (!rc) *out = (float)host[0];
    return rc;
}

}  // extern "C"

extern "C" int admm_cg_solve(const ladmm_operator* op, const ladmm_params* p, int cg_iters, float* x, float* v,
                             float* u, float* residuals, void* stream) {
    OpView ov;
    int rc = check_operator(op, true, "admm_cg_solve", &ov);
    if (rc) return rc;
    if (op->kind != LADMM_OP_SR) return fail(DSNLM_EINVAL, "admm_cg_solve: super-resolution operator only");
    float h;
    rc = check_params(p, op->n1, op->n2, "admm_cg_solve", &h);
    if (rc) return rc;
    if (cg_iters < 0) return fail(DSNLM_EINVAL, "admm_cg_solve: cg_iters must be >= 0");
    if (!x || !v || !u) return fail(DSNLM_EINVAL, "admm_cg_solve: null pointer");
    if (p->iters == 0) return DSNLM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    dsnlm_weights* w = nullptr;
    rc = prepare_handle(op->n1, op->n2, p->S, p->P, h, &w);
    if (rc) return rc;
    float *lr, *partials;
    rc = ensure_solver_scratch(w, ov, op, 1, &lr, &partials);
    const size_t n = (size_t)op->n1 * op->n2;
    const int nb = blocks(n);
    // CG vectors: A^T y, r, p, q (n each) and the device scalars
    float* cgbuf = nullptr;
    if (!rc) rc = check_hip(hipMalloc(&cgbuf, (4 * n + 64) * sizeof(float)), "admm_cg_solve scratch");
    if (rc) {
        dsnlm_weights_destroy(w);
        return rc;
    }
    float* aty = cgbuf;
    float* r = aty + n;
    float* pd = r + n;
    float* q = pd + n;
    CGScalars* sc = reinterpret_cast<CGScalars*>(q + n);
    {
        ProfScope prof(DSNLM_K_LADMM, st);
        StepScalars s{};
        launch_sr_adjoint(ov.g, ov.taps, op->boundary, op->y, aty, nullptr, nullptr, nullptr, s, 0, st);
        rc = check_hip(hipGetLastError(), "A^T y");
    }
    for (int k = 1; k <= p->iters && !rc; ++k) {
        {
            ProfScope prof(DSNLM_K_LADMM, st);
            enqueue_AtA(op, ov, x, lr, q, st);
            hipLaunchKernelGGL(k_cg_start, dim3(nb), dim3(256), 0, st, aty, q, x, v, u, r, pd, p->rho, (int)n,
                               partials);
            hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(256), 0, st, partials, nb, sc, 0);
            for (int it = 0; it < cg_iters; ++it) {
                enqueue_AtA(op, ov, pd, lr, q, st);
                hipLaunchKernelGGL(k_cg_pq, dim3(nb), dim3(256), 0, st, pd, q, p->rho, (int)n, partials);
                hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(256), 0, st, partials, nb, sc, 1);
                hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(256), 0, st, x, r, pd, q, sc, (int)n, partials);
                hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(256), 0, st, partials, nb, sc, 2);
                hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(256), 0, st, r, pd, sc, (int)n);
            }
            hipLaunchKernelGGL(k_add, dim3(nb), dim3(256), 0, st, x, u, w->zbuf, (int)n);
            rc = check_hip(hipGetLastError(), "conjugate gradients");
        }
        if (!rc) rc = enqueue_denoise_dual(p, k, w, x, v, u, partials, residuals != nullptr, nullptr, st);
        if (!rc && residuals)
            rc = enqueue_residuals(partials, op->n1, op->n2, 1, p->rho, residuals + 2 * (size_t)(k - 1), st);
    }
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "admm_cg_solve synchronise");
    (void)hipFree(cgbuf);
    dsnlm_weights_destroy(w);
    return rc;
}
