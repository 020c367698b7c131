// Half-window form of the accumulating sweeps (pass A, the pass-B family and
// the backward sweep C) on gfx950.
//
// The kernel weight of a pair is symmetric, a_{s,s+d} = a_{s+d,s}: the hat
// Lambda_d is even in d and D_{s,d} = D_{s+d,-d} (Section 3, the patch
// distance and eq. for a).  So every unordered pair {s, r = s + d} is
// evaluated once, for the shifts of a half window H = {dy > 0} u {dy = 0,
// dx > 0}; d = 0 (a = 1) is added analytically.  Each sweep sums, for every
// pixel, a times a per-pixel factor of the partner:
//
//   pass A       sum_r a                       (omega)
//   pass B, apply sum_r a c_r, sum_r a c_r x_r  (delta, B')
//   sweep C      sum_r a t_r, sum_r a w_r      (backward)
//   plain NLM    sum_r k, sum_r k x_r          (eq. NLM: no hat, y = ratio)
//
// A tile adds a * factor(r) to its own pixel s in registers and a * factor(s)
// to the partner r in an LDS accumulator that spans the tile's partner region
// (S rows below, S columns either side), next to the partner factors.  The
// guide is read from a mirrored copy in memory (made before pass A) rather
// than staged in LDS, which keeps the LDS at two tiles per CU.  The region is written to a
// per-tile partial buffer, and a gather kernel adds for every pixel the
// regions of the (at most six) tiles covering it, in a fixed order, then the
// d = 0 term, and finishes the pass exactly as the full-window sweep does.
// The sums are the same as the full window's, up to the order of the FP32
// additions.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "sr_step.h"

namespace dsnlm {

namespace {


template <int P, int S_CLASS, int GW_ = 11>
struct HGeo {
    static constexpr int TH = 32, TW = 64;   // s-tile (the forward tiling)
    // phase-1 strip height: 8 rows; 16 for wide patches, whose strips would
    // otherwise spend most of their work restarting the sliding sum
    static constexpr int R = P > kMaxP ? 16 : 8;
    static constexpr int L = 4;              // outputs per thread
    static constexpr int NT = TH * (TW / L);  // 512 threads
    static constexpr int TWE = TW + 2 * P;
    static constexpr int NITEM1 = TWE * (TH / R);
    static constexpr int GWIN = GW_;   // shifts per register window (one dx, consecutive dy)
    // partner region: rows ti0 .. ti0+TH+S, columns tj0-S .. tj0+TW+S (odd stride)
    static constexpr int AW = (TW + 2 * S_CLASS) | 1;
    static constexpr int VW0 = ((TWE + 3) / 4) * 4;
    static constexpr int VW = ((VW0 / 4) % 2) ? VW0 : VW0 + 4;
    static_assert(NITEM1 <= NT, "one phase-1 item per thread");
};

// floats per partner-region entry in LDS: the sum of a (pass A); the partner
// factor c x and the sum of a c x (the apply of built weights, whose sum of
// a c is fixed with the weights: the gather takes it as delta / c); or the
// partner factors and the two factor-weighted sums (the others)
constexpr int half_nc(int mode) { return mode == kPassA ? 1 : mode == kApply ? 2 : 4; }
// channels of the partial buffer
constexpr int half_np(int mode) { return mode == kPassA || mode == kApply ? 1 : 2; }

template <int P, int S_CLASS>
size_t half_lds_floats(int S, int mode) {
    using G = HGeo<P, S_CLASS>;
    return (size_t)2 * G::TH * G::VW + (size_t)(G::TH + S) * G::AW * half_nc(mode);
}

__device__ __forceinline__ int reflect_h(int k, int n) {
    if (k < 0) k = -k - 1;
    if (k >= n) k = 2 * n - 1 - k;
    k = k < 0 ? 0 : k;
    k = k >= n ? n - 1 : k;
    return k;
}

// Shift number f (0 <= f < 2S(S+1)) of the half window H = {dy > 0} u {dy = 0,
// dx > 0} in the order dx ascending, dy ascending: the S(S+1) shifts with
// dx <= 0 (dy = 1..S), then those with dx > 0 (dy = 0..S).  Needs S >= 1.
__device__ __forceinline__ void half_shift(int f, int S, int& dx, int& dy) {
    if (f < S * (S + 1)) {
        dx = -S + f / S;
        dy = 1 + f % S;
    } else {
        const int g = f - S * (S + 1);
        dx = 1 + g / (S + 1);
        dy = g % (S + 1);
    }
}

// the tile's index within its image
__device__ __forceinline__ int local_tile(int ti0, int tj0, int n2, int TH, int TW) {
    const int ntx = (n2 + TW - 1) / TW;
    return (ti0 / TH) * ntx + tj0 / TW;
}

// The guide mirrored into a margin of m = S + P on every side, so that the
// sweeps read any patch pixel without index reflection.  One block per
// s-tile writes the tile's rows and columns, plus the margins beside it when
// the tile is on the image border.
template <bool BATCH>
__global__ void __launch_bounds__(256)
k_half_pad(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles, int m) {
    constexpr int TH = 32, TW = 64;
    ImgDesc d;
    int ti0, tj0;
    if constexpr (BATCH) {
        const TileRef t = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
        d = batch[t.img];
        ti0 = t.ti0;
        tj0 = t.tj0;
    } else {
        d = one;
        ti0 = blockIdx.y * TH;
        tj0 = blockIdx.x * TW;
    }
    const int n1 = d.n1, n2 = d.n2, W2 = n2 + 2 * m;
    const int i0 = ti0 == 0 ? -m : ti0;
    const int i1 = ti0 + TH >= n1 ? n1 + m : ti0 + TH;
    const int j0 = tj0 == 0 ? -m : tj0;
    const int j1 = tj0 + TW >= n2 ? n2 + m : tj0 + TW;
    const int w = j1 - j0;
    for (int e = threadIdx.x; e < (i1 - i0) * w; e += 256) {
        const int i = i0 + e / w, j = j0 + e % w;
        d.zpad[(size_t)(i + m) * W2 + j + m] = d.z[(size_t)reflect_h(i, n1) * n2 + reflect_h(j, n2)];
    }
}

// Pass A carries fewer live values: its registers are capped so that three
// tiles share a CU (its LDS allows it).
template <int P, int S_CLASS, int MODE, bool BATCH>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MODE == kPassA && P < 5 ? 6 : 1)))
k_half(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles, int S,
       HatTable hat, int ngrp) {
    // window length by measurement on gfx950 (pass A: 15, the others: 11; at
    // S = 10 either covers every dy of a dx in one group)
    using G = HGeo<P, S_CLASS, MODE == kPassA ? 15 : 11>;
    constexpr int NT = G::NT, TH = G::TH, TW = G::TW, R = G::R, L = G::L;
    constexpr int AW = G::AW, VW = G::VW;
    constexpr int NC = half_nc(MODE);
    constexpr int NE = R + 2 * P;
    extern __shared__ __align__(16) float lds[];
    const int tid = threadIdx.x;

    ImgDesc d;
    int ti0, tj0;
    bool first;
    if constexpr (BATCH) {
        const TileRef t = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
        d = batch[t.img];
        ti0 = t.ti0;
        tj0 = t.tj0;
        first = (t.flags & 1) != 0;
    } else {
        d = one;
        ti0 = blockIdx.y * TH;
        tj0 = blockIdx.x * TW;
        first = blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0;
    }
    // dx group of this block (a single-image launch may split the half
    // window's dx range over blockIdx.z; each group has its own regions)
    const int grp = BATCH ? 0 : (int)blockIdx.z;
    // this block's shifts: a contiguous range of the half window in the order
    // dx ascending, dy ascending within a dx (a single-image launch may split
    // the 2S(S+1) shifts into ngrp ranges of equal length, one per blockIdx.z;
    // each group has its own regions).  (dxF, dyF) .. (dxL, dyL): the first
    // and last shift (inclusive); empty when dxF > dxL.
    int dxF = 1, dyF = 0, dxL = 0, dyL = 0;
    {
        const int H = 2 * S * (S + 1);
        const int f0 = BATCH ? 0 : (int)((long long)grp * H / ngrp);
        const int f1 = BATCH ? H : (int)((long long)(grp + 1) * H / ngrp);
        if (f1 > f0) {
            half_shift(f0, S, dxF, dyF);
            half_shift(f1 - 1, S, dxL, dyL);
        }
    }
    const int n1 = d.n1, n2 = d.n2;
    const int AH = TH + S, AWr = TW + 2 * S;
    float* Vb = lds;
    float* Acc = lds + 2 * TH * VW;  // partner region, NC floats per entry

    // ---- the partner region: factors (c, c x) or (t, w) and zeroed sums.
    // The loop has a compile-time trip count (the region of the largest S of
    // the class), so every thread issues all its loads before the first wait.
    constexpr int NINIT = ((TH + S_CLASS) * (TW + 2 * S_CLASS) + NT - 1) / NT;
    if constexpr (NC == 1) {
        for (int idx = tid; idx < AH * AWr; idx += NT) {
            const int r = idx / AWr, q = idx - r * AWr;
            Acc[r * AW + q] = 0.f;
        }
    } else {
        float2 fv[NINIT];
        int slot[NINIT];
#pragma unroll
        for (int it = 0; it < NINIT; ++it) {
            const int idx = tid + it * NT;
            fv[it] = make_float2(0.f, 0.f);
            slot[it] = -1;
            if (idx < AH * AWr) {
                const int r = idx / AWr, q = idx - r * AWr;
                slot[it] = r * AW + q;
                const int gi = ti0 + r, gj = tj0 - S + q;
                if ((unsigned)gi < (unsigned)n1 && (unsigned)gj < (unsigned)n2) {
                    const size_t p = (size_t)gi * n2 + gj;
                    if constexpr (MODE == kPassC) {
                        fv[it] = reinterpret_cast<const float2*>(d.aux_in)[p];
                    } else if constexpr (MODE == kNLM) {
                        fv[it] = make_float2(1.f, d.x[p]);
                    } else if constexpr (MODE == kPassBBuild) {
                        fv[it] = make_float2(d.c[p], 0.f);
                    } else {
                        fv[it] = make_float2(d.c[p], d.x[p]);  // c x formed below
                    }
                }
            }
        }
#pragma unroll
        for (int it = 0; it < NINIT; ++it) {
            if (slot[it] >= 0) {
                float2 f = fv[it];
                if constexpr (MODE == kPassBApply || MODE == kApply) f.y = f.x * f.y;
                if constexpr (NC == 2)
                    reinterpret_cast<float2*>(Acc)[slot[it]] = make_float2(f.y, 0.f);
                else
                    reinterpret_cast<float4*>(Acc)[slot[it]] = make_float4(f.x, f.y, 0.f, 0.f);
            }
        }
    }
    if constexpr (MODE == kPassA) {
        if (first && tid == 0) *d.key = 0ull;  // the pass-B gather takes the max after this
    }
    if constexpr (MODE == kNLM) {
        // plain NLM has no normalisation by a maximum: store m = 1 so that the
        // common update x + B'/m applies its increment unchanged
        if (first && tid == 0) *d.key = ((unsigned long long)__float_as_uint(1.0f) << 32) | 0xffffffffull;
    }

    // ---- phase-1 item: one column strip of R rows (threads past NITEM1 idle).
    // The guide comes from its mirrored copy in memory; lanes walk along
    // columns, so each load of a wave reads one contiguous row segment.  The
    // range check returns zeros past the copy (only masked outputs see them).
    const int m = S + P, W2 = n2 + 2 * m;
    const bool has1 = tid < G::NITEM1;
    const int it = has1 ? tid : 0;
    const int strip = it / G::TWE;
    const int c1 = it - strip * G::TWE;
    // mirrored copy: pixel (i, j) at (i + m) * W2 + j + m; the strip's first
    // reference pixel is (ti0 - P + strip R, tj0 - P + c1)
    const int zbase = (ti0 + S + strip * R) * W2 + tj0 + S + c1;
    const size_t zbytes = (size_t)(n1 + 2 * m) * W2 * 4;
    const __amdgpu_buffer_rsrc_t zrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(d.zpad), (short)0, (int)(zbytes < 0x7ffffff0u ? zbytes : 0x7ffffff0u), 0x00020000);
    auto zload = [&](int off) { return __builtin_amdgcn_raw_buffer_load_b32(zrs, off * 4, 0, 0); };
    const int voff = strip * R * VW + c1;
    float ref[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) ref[q] = __builtin_bit_cast(float, zload(zbase + q * W2));

    const int pi = tid % TH;
    // a wave holds two column groups 32 apart: with odd row strides its scalar
    // LDS accesses then hit 64 distinct banks
    const int pj = ((tid / TH) & 1) * (TW / 2) + (tid / (2 * TH)) * L;
    const int own = pi * AW + pj + S;  // own pixel in the partner region
    __syncthreads();
    float acc0[L], acc1[L], f0[L], f1[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        acc0[k] = 0.f;
        acc1[k] = 0.f;
        if constexpr (NC == 4) {
            const float4 v = reinterpret_cast<const float4*>(Acc)[own + k];
            f0[k] = v.x;
            f1[k] = v.y;
        } else if constexpr (NC == 2) {
            f0[k] = 0.f;
            f1[k] = reinterpret_cast<const float2*>(Acc)[own + k].x;
        } else {
            f0[k] = 0.f;
            f1[k] = 0.f;
        }
    }
    const float beta = d.beta;
    const int gi_own = ti0 + pi, gj_own = tj0 + pj;
    const bool s_in = ti0 + TH <= n1 && tj0 + TW <= n2;

    constexpr int NV = ((L + 2 * P + 3) / 4) * 4;
    constexpr int GW = G::GWIN;
    constexpr int NW = NE + GW - 1;
    // The shifted rows of a group of shifts (one dx, GW consecutive dy) are
    // loaded one group ahead, so their latency is spent on the group before;
    // pass A (registers capped) and patches above 7x7 (past 128 registers,
    // one tile per CU) have none to spare and load each group's rows at its
    // start.
    constexpr bool PF = MODE != kPassA && P <= 3;
    // With the look-ahead, only the threads with a phase-1 item load windows
    // (the others, the last three waves of the block and part of the fifth,
    // would only repeat item 0's loads).
    float nwin[PF ? NW : 1];
    if constexpr (PF) {
#pragma unroll
        for (int q = 0; q < NW; ++q) nwin[q] = 0.f;
        if (has1) {
            const int zw = zbase + dyF * W2 + dxF;
#pragma unroll
            for (int q = 0; q < NW; ++q) nwin[q] = __builtin_bit_cast(float, zload(zw + q * W2));
        }
    }
    int t = 0;
    for (int dx = dxF; dx <= dxL; ++dx) {
        const int dyA = dx == dxF ? dyF : (dx > 0 ? 0 : 1);  // the half window
        const int dyB = dx == dxL ? dyL : S;
        // log2 of the hat's dx factor in a vector register (a VALU
        // instruction reads one scalar operand, so log2 Lambda_d is then one
        // addition per shift instead of a move and an addition)
        float lgx;
        asm("v_mov_b32 %0, %1" : "=v"(lgx) : "s"(hat.lg[dx + S]));
        for (int dy0 = dyA; dy0 <= dyB; dy0 += GW) {
            float win[NW];
            if constexpr (PF) {
#pragma unroll
                for (int q = 0; q < NW; ++q) win[q] = nwin[q];
                // the next group; past the last one this is an unused read,
                // inside the range-checked buffer
                const int ndx = dy0 + GW <= dyB ? dx : dx + 1;
                const int ndy0 = dy0 + GW <= dyB ? dy0 + GW : (ndx > 0 ? 0 : 1);
                if (has1) {
                    const int zw = zbase + ndy0 * W2 + ndx;
#pragma unroll
                    for (int q = 0; q < NW; ++q) nwin[q] = __builtin_bit_cast(float, zload(zw + q * W2));
                }
            } else {
                // (unguarded: under pass A's register cap the guarded form
                // spills)
                const int zw = zbase + dy0 * W2 + dx;
#pragma unroll
                for (int q = 0; q < NW; ++q) win[q] = __builtin_bit_cast(float, zload(zw + q * W2));
            }
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                const int dy = dy0 + g;
                if (dy <= dyB) {
                    float* V = Vb + (t & 1) * (TH * VW);
                    // read here, so that the scalar load has returned by the
                    // barrier and no wait for it holds up the LDS reads after it
                    const float lg = hat.lg[dy + S] + lgx;
                    // phase 1: vertical sliding box of (z(p) - z(p+d))^2.
                    // Issue priorities: phase 1 highest (the block's barrier
                    // waits for it while the other block on the CU is in
                    // phase 2), then the LDS reads that open phase 2, then
                    // the rest.  Measured on the 64-image batch against no
                    // priorities: pass A -5%, pass B and sweep C -5%.
                    __builtin_amdgcn_s_setprio(2);
                    if (has1) {
                        float tq[NE];
#pragma unroll
                        for (int q = 0; q < NE; ++q) tq[q] = ref[q] - win[g + q];
                        float v = tq[0] * tq[0];
#pragma unroll
                        for (int q = 1; q <= 2 * P; ++q) v = fmaf(tq[q], tq[q], v);
                        float* vo = V + voff;
                        vo[0] = v;
#pragma unroll
                        for (int q = 1; q < R; ++q) {
                            v = fmaf(tq[q + 2 * P], tq[q + 2 * P], v);
                            v = fmaf(-tq[q - 1], tq[q - 1], v);
                            vo[q * VW] = v;
                        }
                    }
                    __builtin_amdgcn_s_setprio(1);
                    __syncthreads();
                    // phase 2: horizontal sliding box, weights, both-sided sums
                    float vv[NV];
                    {
                        const float* vr = V + pi * VW + pj;
#pragma unroll
                        for (int q = 0; q < NV / 4; ++q) {
                            const float4 t4 = reinterpret_cast<const float4*>(vr)[q];
                            vv[4 * q + 0] = t4.x;
                            vv[4 * q + 1] = t4.y;
                            vv[4 * q + 2] = t4.z;
                            vv[4 * q + 3] = t4.w;
                        }
                    }
                    // the partner entries, read before the weights so that
                    // the exponentials cover the read latency (the entries
                    // of one shift are distinct across the block)
                    const int pr = own + dy * AW + dx;  // partner entry of output 0
                    float4 pv[NC == 4 ? L : 1];
                    float2 pv2[NC == 2 ? L : 1];
                    if constexpr (NC == 4) {
#pragma unroll
                        for (int k = 0; k < L; ++k) pv[k] = reinterpret_cast<const float4*>(Acc)[pr + k];
                    } else if constexpr (NC == 2) {
#pragma unroll
                        for (int k = 0; k < L; ++k) pv2[k] = reinterpret_cast<const float2*>(Acc)[pr + k];
                    }
                    __builtin_amdgcn_s_setprio(0);
                    float hs = vv[0];
#pragma unroll
                    for (int q = 1; q <= 2 * P; ++q) hs += vv[q];
                    float a[L];
                    a[0] = __builtin_amdgcn_exp2f(lg - beta * hs);
#pragma unroll
                    for (int k = 1; k < L; ++k) {
                        hs += vv[k + 2 * P] - vv[k - 1];
                        a[k] = __builtin_amdgcn_exp2f(lg - beta * hs);
                    }
                    const bool inside = s_in && ti0 + TH - 1 + dy < n1 && tj0 + dx >= 0 &&
                                        tj0 + TW - 1 + dx < n2;
                    if (!inside) {
                        const bool rowok = gi_own < n1 && gi_own + dy < n1;
#pragma unroll
                        for (int k = 0; k < L; ++k) {
                            const int gj = gj_own + k;
                            const bool ok = rowok && gj < n2 && (unsigned)(gj + dx) < (unsigned)n2;
                            a[k] = ok ? a[k] : 0.f;
                        }
                    }
                    if constexpr (NC == 1) {
#pragma unroll
                        for (int k = 0; k < L; ++k) {
                            acc0[k] += a[k];
                            Acc[pr + k] += a[k];
                        }
                    } else if constexpr (NC == 2) {
#pragma unroll
                        for (int k = 0; k < L; ++k) {
                            acc1[k] = fmaf(a[k], pv2[k].x, acc1[k]);
                            Acc[2 * (pr + k) + 1] = fmaf(a[k], f1[k], pv2[k].y);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < L; ++k) {
                            float4* e = reinterpret_cast<float4*>(Acc) + pr + k;
                            const float4 v = pv[k];
                            acc0[k] = fmaf(a[k], v.x, acc0[k]);
                            acc1[k] = fmaf(a[k], v.y, acc1[k]);
                            reinterpret_cast<float2*>(e)[1] =
                                make_float2(fmaf(a[k], f0[k], v.z), fmaf(a[k], f1[k], v.w));
                        }
                    }
                    ++t;
                }
            }
        }
    }
    // the last shift's partner updates are complete after this barrier; then
    // the own-pixel sums join the region (each thread owns its entries)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < L; ++k) {
        if constexpr (NC == 1) {
            Acc[own + k] += acc0[k];
        } else if constexpr (NC == 2) {
            Acc[2 * (own + k) + 1] += acc1[k];
        } else {
            float2* e = reinterpret_cast<float2*>(reinterpret_cast<float4*>(Acc) + own + k) + 1;
            const float2 v = *e;
            *e = make_float2(v.x + acc0[k], v.y + acc1[k]);
        }
    }
    __syncthreads();
    const size_t reg = (size_t)AH * AWr;
    const int lt = local_tile(ti0, tj0, n2, TH, TW);
    const size_t ntl = (size_t)((n1 + TH - 1) / TH) * ((n2 + TW - 1) / TW);
    float* part = (grp == 0 ? d.part : d.gpart + (grp - 1) * ntl * reg * half_np(MODE)) +
                  (size_t)lt * reg * half_np(MODE);
    for (int idx = tid; idx < AH * AWr; idx += NT) {
        const int r = idx / AWr, q = idx - r * AWr;
        if constexpr (NC == 1) {
            part[idx] = Acc[r * AW + q];
        } else if constexpr (NC == 2) {
            part[idx] = Acc[2 * (r * AW + q) + 1];
        } else {
            const float4 v = reinterpret_cast<const float4*>(Acc)[r * AW + q];
            reinterpret_cast<float2*>(part)[idx] = make_float2(v.z, v.w);
        }
    }
}

__device__ __forceinline__ unsigned long long wave_max_u64_h(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Threads of a gather block: 256 for a batch tile (32 x 64 pixels), 512 for a
// quarter tile of a single image (8 x 64 pixels, one per thread, so that no
// thread waits on a second pixel's loads).
constexpr int gather_threads(bool batch) { return batch ? 256 : 512; }

// One block per s-tile: every pixel of the tile sums the partial regions of
// the tiles covering it (own, left, right, above, above-left, above-right),
// adds the d = 0 term and finishes the pass.
template <int MODE, bool BATCH>
__global__ void __launch_bounds__(512)
k_half_gather(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles, int S,
              int ngrp) {
    constexpr int TH = 32, TW = 64;
    constexpr int NT = gather_threads(BATCH), NW = NT / 64;
    constexpr int NP = half_np(MODE);
    ImgDesc d;
    int ti0, tj0;
    if constexpr (BATCH) {
        const TileRef t = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
        d = batch[t.img];
        ti0 = t.ti0;
        tj0 = t.tj0;
    } else {
        d = one;
        ti0 = blockIdx.y * TH;
        tj0 = blockIdx.x * TW;
    }
    const int n1 = d.n1, n2 = d.n2;
    const int AWr = TW + 2 * S;
    const size_t reg = (size_t)(TH + S) * AWr;
    const int ntx = (n2 + TW - 1) / TW;
    const int lt = (ti0 / TH) * ntx + tj0 / TW;
    const int tx = tj0 / TW;
    const size_t ntl = (size_t)((n1 + TH - 1) / TH) * ntx;
    unsigned long long best = 0ull;
    // a single-image launch splits the tile's rows over gridDim.z blocks
    const int rows = TH / (int)gridDim.z, li0 = (int)blockIdx.z * rows;
    float m = 1.f;
    if constexpr (MODE == kApply) m = __uint_as_float((unsigned)(*d.key >> 32));  // the built weights' m
    float rp = 0.f, rd = 0.f;  // fused dual half: residual sums of this thread
    // the next iteration's x-step (single image, lstep set): its window loads
    // go out with the partial loads; the thread's one pixel keeps x, v and u
    using XW = SRWindow<kNextStepRows, TW, NT>;
    XW xwin;
    float kx = 0.f, kv = 0.f, ku = 0.f;
    bool kin = false;
    if constexpr (MODE == kApply && !BATCH)
        if (d.lstep) xwin.load(d.lx, d.lstep->y, d.lstep->g, ti0 + li0, tj0, threadIdx.x);
    for (int e = threadIdx.x; e < rows * TW; e += NT) {
        const int li = li0 + e / TW, lj = e % TW;
        const int gi = ti0 + li, gj = tj0 + lj;
        if (gi >= n1 || gj >= n2) continue;
        float s0 = 0.f, s1 = 0.f;
        // the regions covering the pixel (own, left, right, above, above-left,
        // above-right) and the dx groups of each: all loads are issued first,
        // then added in that fixed order (regions, and groups within each)
        const bool left = tx > 0 && lj < S, right = tx + 1 < ntx && lj >= TW - S;
        const bool above = ti0 > 0 && li < S;
        const int up = lt - ntx;
        size_t off[6];
        bool ok[6];
        off[0] = (size_t)lt * reg + (size_t)li * AWr + lj + S;
        off[1] = (size_t)(lt - 1) * reg + (size_t)li * AWr + lj + TW + S;
        off[2] = (size_t)(lt + 1) * reg + (size_t)li * AWr + lj - TW + S;
        off[3] = (size_t)up * reg + (size_t)(li + TH) * AWr + lj + S;
        off[4] = (size_t)(up - 1) * reg + (size_t)(li + TH) * AWr + lj + TW + S;
        off[5] = (size_t)(up + 1) * reg + (size_t)(li + TH) * AWr + lj - TW + S;
        ok[0] = true;
        ok[1] = left;
        ok[2] = right;
        ok[3] = above;
        ok[4] = above && left;
        ok[5] = above && right;
        constexpr int GMAX = BATCH ? 1 : kMaxShiftGroups;  // a batch never splits
        float2 val[6][GMAX];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
#pragma unroll
            for (int g = 0; g < GMAX; ++g) {
                val[r][g] = make_float2(0.f, 0.f);
                if (ok[r] && g < ngrp) {
                    const float* src = g == 0 ? d.part : d.gpart + (g - 1) * ntl * reg * NP;
                    if constexpr (NP == 1) val[r][g].x = src[off[r]];
                    else val[r][g] = reinterpret_cast<const float2*>(src)[off[r]];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
#pragma unroll
            for (int g = 0; g < GMAX; ++g) {
                if (ok[r] && g < ngrp) {
                    s0 += val[r][g].x;
                    if constexpr (NP == 2) s1 += val[r][g].y;
                }
            }
        }
        const size_t p = (size_t)gi * n2 + gj;
        if constexpr (MODE == kPassA) {
            d.c[p] = 1.0f / sqrtf(s0 + 1.0f);  // omega includes a_{s,s} = 1
        } else if constexpr (MODE == kPassC) {
            const float2 tw = reinterpret_cast<const float2*>(d.aux_in)[p];
            reinterpret_cast<float2*>(d.aux_out)[p] = make_float2(s0 + tw.x, s1 + tw.y);
        } else if constexpr (MODE == kNLM) {
            // d = 0: k = 1.  y = sum k x_r / sum k = x + (sum k x_r - x sum k) / sum k
            const float xs = d.x[p];
            s0 += 1.f;
            s1 += xs;
            const float inc = (s1 - xs * s0) / s0;
            d.bp[p] = inc;
            if (d.y) d.y[p] = xs + inc;
        } else {
            const float cs = d.c[p];
            if constexpr (MODE == kApply) {
                // the one channel is sum_r a c_r x_r; sum_r a c_r (d = 0
                // included) is fixed with the weights: pass B's own sum, or
                // delta / c where the build kept none
                s1 = s0;
                s0 = d.s0 ? d.s0[p] : d.delta[p] / cs;
            } else {
                s0 += cs;  // d = 0: a = 1, partner factor c_s
                if constexpr (!BATCH && (MODE == kPassBApply || MODE == kPassBBuild))
                    if (d.s0) d.s0[p] = s0;
            }
            if constexpr (MODE == kPassBApply || MODE == kApply) {
                const float xs = d.x[p];
                s1 += cs * xs;
                const float bp = cs * (s1 - xs * s0);
                d.bp[p] = bp;
                if constexpr (MODE == kApply) {
                    const float vn = xs + bp / m;  // y = W x
                    if (d.y) d.y[p] = vn;
                    if (d.lu) {
                        // Algorithm 1, dual half: u <- u + x - v, v <- W z
                        const float xv = d.lx[p], vo = d.lv[p];
                        const float un = d.lu[p] + xv - vn;
                        d.lu[p] = un;
                        d.lv[p] = vn;
                        kx = xv;
                        kv = vn;
                        ku = un;
                        kin = true;
                        rp = fmaf(xv - vn, xv - vn, rp);
                        rd = fmaf(vn - vo, vn - vo, rd);
                    }
                }
            }
            if constexpr (MODE == kPassBApply || MODE == kPassBBuild) {
                const float dl = cs * s0;
                d.delta[p] = dl;
                const unsigned long long kk =
                    ((unsigned long long)__float_as_uint(dl) << 32) | (unsigned long long)(~(unsigned)p);
                best = kk > best ? kk : best;
            }
        }
    }
    if constexpr (MODE == kApply) {
        if (d.lres) {
            // fixed-order block sums of the residual terms (wave, then block)
            __shared__ float wsum[2][NW];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                rp += __shfl_xor(rp, off, 64);
                rd += __shfl_xor(rd, off, 64);
            }
            if ((threadIdx.x & 63) == 0) {
                wsum[0][threadIdx.x >> 6] = rp;
                wsum[1][threadIdx.x >> 6] = rd;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                const int b = ((int)blockIdx.z * (int)gridDim.y + (int)blockIdx.y) * (int)gridDim.x + (int)blockIdx.x;
                float r2[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    r2[c] = (wsum[c][0] + wsum[c][1]) + (wsum[c][2] + wsum[c][3]);
                    if constexpr (NW == 8)
                        r2[c] = r2[c] + ((wsum[c][4] + wsum[c][5]) + (wsum[c][6] + wsum[c][7]));
                }
                d.lres[2 * b] = r2[0];
                d.lres[2 * b + 1] = r2[1];
            }
        }
        if constexpr (!BATCH) {
            if (d.lstep) {
                static_assert(BATCH || NT == kNextStepRows * TW, "one pixel per thread");
                const int e = threadIdx.x;
                next_xstep(xwin, d.lstep, ti0 + li0 + e / TW, tj0 + e % TW, kin, kx, kv, ku);
            }
        }
    }
    if constexpr (MODE == kPassBApply || MODE == kPassBBuild) {
        // one atomic per block: wave maxima, then the block's in LDS
        __shared__ unsigned long long wmax[NW];
        best = wave_max_u64_h(best);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long b = wmax[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) b = wmax[w] > b ? wmax[w] : b;
            if (b != 0ull) atomicMax(d.key, b);
        }
    }
}

template <int P, int S_CLASS, int MODE, bool BATCH>
hipError_t half_attr() {
    static bool attr_set = false;  // per instance
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_half<P, S_CLASS, MODE, BATCH>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    return hipSuccess;
}

template <int P, int S_CLASS>
hipError_t half_attr_all() {
    hipError_t e = half_attr<P, S_CLASS, kPassA, false>();
    if (e == hipSuccess) e = half_attr<P, S_CLASS, kPassBApply, false>();
    if (e == hipSuccess) e = half_attr<P, S_CLASS, kPassBBuild, false>();
    if (e == hipSuccess) e = half_attr<P, S_CLASS, kApply, false>();
    if (e == hipSuccess) e = half_attr<P, S_CLASS, kPassC, false>();
    if (e == hipSuccess) e = half_attr<P, S_CLASS, kNLM, false>();
    return e;
}

template <int P>
hipError_t half_prepare_p(int S) {
    return S <= 12 ? half_attr_all<P, 12>() : half_attr_all<P, kMaxS>();
}

template <int P, int S_CLASS, int MODE, bool BATCH>
hipError_t launch_half_one(int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles,
                           hipStream_t st) {
    using G = HGeo<P, S_CLASS>;
    const size_t lds = half_lds_floats<P, S_CLASS>(S, MODE) * sizeof(float);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t ea = half_attr<P, S_CLASS, MODE, BATCH>();
    if (ea != hipSuccess) return ea;
    const dim3 grid = BATCH ? dim3(ntiles) : dim3((one.n2 + G::TW - 1) / G::TW, (one.n1 + G::TH - 1) / G::TH);
    const int ngrp = (BATCH || one.groups < 2 || !one.gpart)
                         ? 1
                         : std::min(std::min(one.groups, std::max(2 * S * (S + 1), 1)), kMaxShiftGroups);
    const dim3 sgrid(grid.x, grid.y, ngrp);
    HatTable hat = make_hat(S);
    if constexpr (MODE == kNLM)
        for (float& v : hat.lg) v = 0.f;  // eq. NLM has no hat
    if constexpr (MODE == kPassA || MODE == kNLM) {  // the mirrored guide copy read by the half sweeps
        ProfScope prof(DSNLM_K_HALF_AUX, st);
        hipLaunchKernelGGL((k_half_pad<BATCH>), grid, dim3(256), 0, st, one, batch, tiles, S + P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        constexpr int kind = MODE == kPassA ? DSNLM_K_PASS_A
                             : (MODE == kPassBApply || MODE == kPassBBuild || MODE == kNLM) ? DSNLM_K_PASS_B
                             : MODE == kApply ? DSNLM_K_APPLY
                                              : DSNLM_K_PASS_C;
        ProfScope prof(kind, st);
        hipLaunchKernelGGL((k_half<P, S_CLASS, MODE, BATCH>), sgrid, dim3(G::NT), lds, st, one, batch, tiles, S,
                           hat, ngrp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope prof(DSNLM_K_HALF_AUX, st);
    const dim3 ggrid(grid.x, grid.y, BATCH ? 1 : kGatherSplit);
    hipLaunchKernelGGL((k_half_gather<MODE, BATCH>), ggrid, dim3(gather_threads(BATCH)), 0, st, one, batch, tiles,
                       S, ngrp);
    return hipGetLastError();
}

template <int P, int S_CLASS, bool BATCH>
hipError_t half_mode(int mode, int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                     int ntiles, hipStream_t st) {
    if constexpr (P > kMaxP) {
        // wide patches: the single-image forward sweeps only
        switch (mode) {
            case kPassA: return launch_half_one<P, S_CLASS, kPassA, false>(S, one, batch, tiles, ntiles, st);
            case kPassBApply: return launch_half_one<P, S_CLASS, kPassBApply, false>(S, one, batch, tiles, ntiles, st);
            case kPassBBuild: return launch_half_one<P, S_CLASS, kPassBBuild, false>(S, one, batch, tiles, ntiles, st);
            case kApply: return launch_half_one<P, S_CLASS, kApply, false>(S, one, batch, tiles, ntiles, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (mode) {
        case kPassA: return launch_half_one<P, S_CLASS, kPassA, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassBApply: return launch_half_one<P, S_CLASS, kPassBApply, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassBBuild: return launch_half_one<P, S_CLASS, kPassBBuild, BATCH>(S, one, batch, tiles, ntiles, st);
        case kApply: return launch_half_one<P, S_CLASS, kApply, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassC: return launch_half_one<P, S_CLASS, kPassC, BATCH>(S, one, batch, tiles, ntiles, st);
        case kNLM: return launch_half_one<P, S_CLASS, kNLM, BATCH>(S, one, batch, tiles, ntiles, st);
        default: return hipErrorInvalidValue;
    }
}

template <int P, bool BATCH>
hipError_t half_s(int mode, int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles,
                  hipStream_t st) {
    if (S <= 12) return half_mode<P, 12, BATCH>(mode, S, one, batch, tiles, ntiles, st);
    return half_mode<P, kMaxS, BATCH>(mode, S, one, batch, tiles, ntiles, st);
}

template <bool BATCH>
hipError_t half_p(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                  int ntiles, hipStream_t st) {
    switch (P) {
        case 0: return half_s<0, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 1: return half_s<1, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 2: return half_s<2, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 3: return half_s<3, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 4: return half_s<4, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 5: return half_s<5, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        default: break;
    }
    if constexpr (!BATCH) {  // wide patches (single image, forward sweeps)
        switch (P) {
            case 6: return half_s<6, false>(mode, S, one, batch, tiles, ntiles, st);
            case 7: return half_s<7, false>(mode, S, one, batch, tiles, ntiles, st);
            case 8: return half_s<8, false>(mode, S, one, batch, tiles, ntiles, st);
            case 9: return half_s<9, false>(mode, S, one, batch, tiles, ntiles, st);
            case 10: return half_s<10, false>(mode, S, one, batch, tiles, ntiles, st);
            case 11: return half_s<11, false>(mode, S, one, batch, tiles, ntiles, st);
            case 12: return half_s<12, false>(mode, S, one, batch, tiles, ntiles, st);
            case 13: return half_s<13, false>(mode, S, one, batch, tiles, ntiles, st);
            case 14: return half_s<14, false>(mode, S, one, batch, tiles, ntiles, st);
            case 15: return half_s<15, false>(mode, S, one, batch, tiles, ntiles, st);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

// floats before the mirrored guide: the half-window partial regions, or for
// wide patches the wide passes' group sums if those are larger
static size_t part_regions(int n1, int n2, int S, int P) {
    const size_t tiles = (size_t)((n1 + 31) / 32) * ((n2 + 63) / 64);
    size_t regions = tiles * (size_t)(32 + S) * (64 + 2 * S) * 2;
    if (P > kMaxP) regions = std::max(regions, wide_part_floats(n1, n2, S));
    return (regions + 63) & ~(size_t)63;
}

int half_split_groups(int n1, int n2, int S, int P) {
    const int H = std::max(2 * S * (S + 1), 1);  // shifts of the half window
    int g = tuned_shift_groups(n1, n2, S, P);
    if (g < 1) {
        // default by the number of 32 x 64 tiles, from timings of the forward
        // and a frozen apply on MI355X (S = 7 and 10): 8 groups up to 64
        // tiles (256 x 256), 4 up to 256 (512 x 512 is 128), 3 up to 512
        // (1024 x 1024), then 1
        const int tiles = ((n1 + 31) / 32) * ((n2 + 63) / 64);
        g = tiles <= 64 ? 8 : tiles <= 256 ? 4 : tiles <= 512 ? 3 : 1;
    }
    return std::max(1, std::min(std::min(g, H), kMaxShiftGroups));
}

size_t half_group_floats(int n1, int n2, int S, int groups) {
    const size_t tiles = (size_t)((n1 + 31) / 32) * ((n2 + 63) / 64);
    return groups > 1 ? (size_t)(groups - 1) * tiles * (32 + S) * (64 + 2 * S) * 2 : 0;
}

size_t half_part_floats(int n1, int n2, int S, int P) {
    const size_t m = (size_t)S + P;
    return part_regions(n1, n2, S, P) + (n1 + 2 * m) * (n2 + 2 * m) + 64;
}

float* half_zpad(float* part, int n1, int n2, int S, int P) { return part + part_regions(n1, n2, S, P); }

bool half_lds_fits(int S, int P, int mode) {
    size_t f = 0;
    switch (P) {
        case 0: f = S <= 12 ? half_lds_floats<0, 12>(S, mode) : half_lds_floats<0, kMaxS>(S, mode); break;
        case 1: f = S <= 12 ? half_lds_floats<1, 12>(S, mode) : half_lds_floats<1, kMaxS>(S, mode); break;
        case 2: f = S <= 12 ? half_lds_floats<2, 12>(S, mode) : half_lds_floats<2, kMaxS>(S, mode); break;
        case 3: f = S <= 12 ? half_lds_floats<3, 12>(S, mode) : half_lds_floats<3, kMaxS>(S, mode); break;
        case 4: f = S <= 12 ? half_lds_floats<4, 12>(S, mode) : half_lds_floats<4, kMaxS>(S, mode); break;
        case 5: f = S <= 12 ? half_lds_floats<5, 12>(S, mode) : half_lds_floats<5, kMaxS>(S, mode); break;
        default:
            // wide patches (forward sweeps): the V buffers grow with P
            if (P > kMaxPWide || mode == kPassC || mode == kNLM) return false;
            f = S <= 12 ? half_lds_floats<kMaxPWide, 12>(S, mode) : half_lds_floats<kMaxPWide, kMaxS>(S, mode);
            break;
    }
    return f * sizeof(float) <= 160 * 1024;
}

bool half_mode_ok(int mode) {
    return mode == kPassA || mode == kPassBApply || mode == kPassBBuild || mode == kApply || mode == kPassC;
}

hipError_t prepare_half(int S, int P) {
    switch (P) {
        case 0: return half_prepare_p<0>(S);
        case 1: return half_prepare_p<1>(S);
        case 2: return half_prepare_p<2>(S);
        case 3: return half_prepare_p<3>(S);
        case 4: return half_prepare_p<4>(S);
        case 5: return half_prepare_p<5>(S);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_half(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                       int ntiles, hipStream_t st) {
    if (batch) return half_p<true>(mode, S, P, one, batch, tiles, ntiles, st);
    return half_p<false>(mode, S, P, one, batch, tiles, ntiles, st);
}

}  // namespace dsnlm
