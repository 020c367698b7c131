// DSG-NLM passes for wide patches (5 < P <= 15, patch sides 13..31), the
// range of Table 1's patch sizes beyond the register-resident sweeps.
//
// The patch distance still comes from box sums, so its cost per pair does not
// grow with N_p (Section 3, the separable box-sum evaluation): per shift d of
// the full window, a 32 x 32 tile forms e_d = (z(p) - z(p+d))^2 over the tile
// widened by P in LDS, box-sums it vertically (column strips) and then
// horizontally (4 outputs per thread), and accumulates the kernel weight
// a = exp2(log2 Lambda_d - beta D) exactly as the first two loops of
// Algorithm 2 need it (the d = 0 term, a = 1, is part of the window):
//
//   pass A        omega_s = sum_r a                 -> c_s = omega_s^(-1/2)
//   pass B        delta_s = c_s sum_r a c_r, B'_s = c_s sum_r a c_r (x_r - x_s)
//   apply         B'_s only (c and m of a previous build)
//
// Runtime S and P, one image per launch, plain full-window schedule: this path
// serves the patch sizes the fast sweeps do not instantiate, not the
// throughput case.  Partners outside the image drop out (border-cut window);
// patch pixels outside the image take the half-sample mirror of the guide.
// A small image would leave most CUs idle, so the dy range of the window is
// split over blockIdx.z; each group writes its per-pixel sums to a partial
// buffer, and a finishing kernel adds the groups in a fixed order and forms
// the pass's outputs.
#include <cmath>

#include "internal.h"

namespace dsnlm {

namespace {

constexpr int WTH = 32, WTW = 32, WNT = 256, WL = 4;

__device__ __forceinline__ int reflect_w(int k, int n) {
    if (k < 0) k = -k - 1;
    if (k >= n) k = 2 * n - 1 - k;
    k = k < 0 ? 0 : k;
    k = k >= n ? n - 1 : k;
    return k;
}

__device__ __forceinline__ unsigned long long wave_max_w(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// LDS floats: guide tile with an S + P halo, the squared-difference plane
// (tile + P halo), its vertical box sums, and for the pass-B family the
// partner factors (c, c x) over the tile + S halo (float2).
size_t wide_lds_floats(int S, int P, int mode) {
    const size_t m = (size_t)S + P;
    size_t n = (WTH + 2 * m) * (WTW + 2 * m);
    n += (size_t)(WTH + 2 * P) * (WTW + 2 * P);
    n += (size_t)WTH * (WTW + 2 * P);
    n = (n + 1) & ~(size_t)1;
    if (mode != kPassA) n += 2 * (size_t)(WTH + 2 * S) * (WTW + 2 * S);
    return n;
}

template <int MODE>
__global__ void __launch_bounds__(WNT) k_wide(ImgDesc d, int S, int P, HatTable hat, int ngrp) {
    extern __shared__ __align__(16) float lds[];
    const int tid = threadIdx.x;
    const int n1 = d.n1, n2 = d.n2;
    const int ti0 = blockIdx.y * WTH, tj0 = blockIdx.x * WTW;
    const int m = S + P;
    const int ZW = WTW + 2 * m, ZH = WTH + 2 * m;
    const int EW = WTW + 2 * P, EH = WTH + 2 * P;
    const int FW = WTW + 2 * S, FH = WTH + 2 * S;
    float* Zs = lds;
    float* E = Zs + ZH * ZW;
    float* V = E + EH * EW;
    float2* F = reinterpret_cast<float2*>(lds + ((ZH * ZW + EH * EW + WTH * EW + 1) & ~1));

    // ---- staging: the mirrored guide, and the partner factors (zero outside)
    for (int idx = tid; idx < ZH * ZW; idx += WNT) {
        const int r = idx / ZW, q = idx - r * ZW;
        Zs[idx] = d.z[(size_t)reflect_w(ti0 - m + r, n1) * n2 + reflect_w(tj0 - m + q, n2)];
    }
    if constexpr (MODE != kPassA) {
        for (int idx = tid; idx < FH * FW; idx += WNT) {
            const int r = idx / FW, q = idx - r * FW;
            const int gi = ti0 - S + r, gj = tj0 - S + q;
            float2 f = make_float2(0.f, 0.f);
            if ((unsigned)gi < (unsigned)n1 && (unsigned)gj < (unsigned)n2) {
                const size_t p = (size_t)gi * n2 + gj;
                const float cc = d.c[p];
                f = make_float2(cc, MODE == kPassBBuild ? 0.f : cc * d.x[p]);
            }
            F[idx] = f;
        }
    }
    __syncthreads();

    const int pi = tid / (WTW / WL), pj = (tid % (WTW / WL)) * WL;  // 4 outputs of one row
    const int gi = ti0 + pi, gj0 = tj0 + pj;
    const float beta = d.beta;
    float acc0[WL], acc1[WL];
#pragma unroll
    for (int k = 0; k < WL; ++k) acc0[k] = acc1[k] = 0.f;
    // vertical-box work item: one column of the widened tile, 8 rows
    const int c2 = tid % EW, sg = tid / EW;
    const bool has2 = tid < 4 * EW;

    const int grp = blockIdx.z;
    const int dylo = -S + grp * (2 * S + 1) / ngrp, dyhi = -S + (grp + 1) * (2 * S + 1) / ngrp;
    for (int dy = dylo; dy < dyhi; ++dy) {
        for (int dx = -S; dx <= S; ++dx) {
            // e_d over the tile widened by P (image rows ti0-P.., columns tj0-P..)
            for (int idx = tid; idx < EH * EW; idx += WNT) {
                const int r = idx / EW, q = idx - r * EW;
                const float* zr = Zs + (r + S) * ZW + q + S;
                const float t = zr[0] - zr[dy * ZW + dx];
                E[idx] = t * t;
            }
            __syncthreads();
            if (has2) {  // vertical sliding box of 2P + 1 rows
                const float* col = E + sg * 8 * EW + c2;
                float* out = V + sg * 8 * EW + c2;
                float v = 0.f;
                for (int u = 0; u <= 2 * P; ++u) v += col[u * EW];
                out[0] = v;
#pragma unroll
                for (int q = 1; q < 8; ++q) {
                    v += col[(q + 2 * P) * EW] - col[(q - 1) * EW];
                    out[q * EW] = v;
                }
            }
            __syncthreads();
            // horizontal sliding box, weights and sums
            const float* vr = V + pi * EW + pj;
            float hs = 0.f;
            for (int u = 0; u <= 2 * P; ++u) hs += vr[u];
            const float lg = hat.lg[dy + S] + hat.lg[dx + S];
            const bool rowok = gi < n1 && (unsigned)(gi + dy) < (unsigned)n1;
#pragma unroll
            for (int k = 0; k < WL; ++k) {
                if (k > 0) hs += vr[k + 2 * P] - vr[k - 1];
                const float a = __builtin_amdgcn_exp2f(lg - beta * hs);
                const int gj = gj0 + k;
                const bool ok = rowok && gj < n2 && (unsigned)(gj + dx) < (unsigned)n2;
                if constexpr (MODE == kPassA) {
                    acc0[k] += ok ? a : 0.f;
                } else {
                    const float2 f = F[(pi + S + dy) * FW + pj + k + S + dx];  // zero outside the image
                    acc0[k] = fmaf(a, f.x, acc0[k]);
                    acc1[k] = fmaf(a, f.y, acc1[k]);
                }
            }
        }
    }

    // ---- this group's per-pixel sums
    if (gi < n1) {
        const size_t n = (size_t)n1 * n2;
        float2* out = reinterpret_cast<float2*>(d.part) + grp * n;
#pragma unroll
        for (int k = 0; k < WL; ++k)
            if (gj0 + k < n2) out[(size_t)gi * n2 + gj0 + k] = make_float2(acc0[k], acc1[k]);
    }
}

// Sum of the groups (fixed order) and the outputs of the pass.
template <int MODE>
__global__ void __launch_bounds__(256) k_wide_finish(ImgDesc d, int ngrp) {
    const size_t n = (size_t)d.n1 * d.n2;
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    const float2* part = reinterpret_cast<const float2*>(d.part);
    unsigned long long best = 0ull;
    if (p < n) {
        float s0 = 0.f, s1 = 0.f;
        for (int g = 0; g < ngrp; ++g) {
            const float2 v = part[g * n + p];
            s0 += v.x;
            s1 += v.y;
        }
        if constexpr (MODE == kPassA) {
            d.c[p] = 1.0f / sqrtf(s0);
        } else {
            const float cs = d.c[p];
            if constexpr (MODE == kPassBApply || MODE == kApply) {
                const float xs = d.x[p];
                d.bp[p] = cs * (s1 - xs * s0);
            }
            if constexpr (MODE == kPassBApply || MODE == kPassBBuild) {
                const float dl = cs * s0;
                d.delta[p] = dl;
                best = ((unsigned long long)__float_as_uint(dl) << 32) | (unsigned long long)(~(unsigned)p);
            }
        }
    }
    if constexpr (MODE == kPassA) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *d.key = 0ull;  // pass B takes the max
    }
    if constexpr (MODE == kPassBApply || MODE == kPassBBuild) {
        __shared__ unsigned long long wmax[4];
        best = wave_max_w(best);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long b = wmax[0];
            for (int w = 1; w < 4; ++w) b = wmax[w] > b ? wmax[w] : b;
            if (b != 0ull) atomicMax(d.key, b);
        }
    }
}

template <int MODE>
hipError_t launch_wide_mode(int S, int P, const ImgDesc& d, hipStream_t st) {
    const size_t lds = wide_lds_floats(S, P, MODE) * sizeof(float);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_wide<MODE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int ngrp = wide_groups(d.n1, d.n2, S);
    const dim3 grid((d.n2 + WTW - 1) / WTW, (d.n1 + WTH - 1) / WTH, ngrp);
    hipLaunchKernelGGL((k_wide<MODE>), grid, dim3(WNT), lds, st, d, S, P, make_hat(S), ngrp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n = (size_t)d.n1 * d.n2;
    hipLaunchKernelGGL((k_wide_finish<MODE>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, ngrp);
    return hipGetLastError();
}

}  // namespace

int wide_groups(int n1, int n2, int S) {
    // enough blocks for two per CU on 256 CUs, at most one dy row per group
    const int tiles = ((n1 + WTH - 1) / WTH) * ((n2 + WTW - 1) / WTW);
    const int g = (512 + tiles - 1) / tiles;
    return g < 1 ? 1 : (g > 2 * S + 1 ? 2 * S + 1 : g);
}

size_t wide_part_floats(int n1, int n2, int S) { return (size_t)wide_groups(n1, n2, S) * n1 * n2 * 2; }

bool wide_fits(int S, int P) {
    return S >= 0 && S <= kMaxS && P > kMaxP && P <= kMaxPWide &&
           wide_lds_floats(S, P, kPassBApply) * sizeof(float) <= 160 * 1024;
}

hipError_t launch_wide(int mode, int S, int P, const ImgDesc& d, hipStream_t st) {
    if (!wide_fits(S, P) || !d.part) return hipErrorInvalidValue;
    const int kind = mode == kPassA ? DSNLM_K_PASS_A : mode == kApply ? DSNLM_K_APPLY : DSNLM_K_PASS_B;
    ProfScope prof(kind, st);
    switch (mode) {
        case kPassA: return launch_wide_mode<kPassA>(S, P, d, st);
        case kPassBApply: return launch_wide_mode<kPassBApply>(S, P, d, st);
        case kPassBBuild: return launch_wide_mode<kPassBBuild>(S, P, d, st);
        case kApply: return launch_wide_mode<kApply>(S, P, d, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dsnlm
