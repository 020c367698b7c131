// Backward sweep D on the forward's tiling: the guide and bandwidth
// gradients of y = W(z, h) x (chain rule through eq. NLM and steps S1-S3).
//
// For a shift d of the half window H (D-bar of a pair is symmetric, so each
// unordered pair is visited once) and the pixels s of a 32 x 64 tile:
//   D-bar(s, d) = -kappa a (abar_{s,d} + abar_{s+d,-d})          (phases 1-2)
//   G(q) = sum over the patch box of D-bar(q - k, d), the part from this
//          tile's s, for q in the tile widened by P on every side  (phases 3-4)
//   T(q) = (z(q) - z(q+d)) G(q):  zbar(q) += 2 T(q),  zbar(q+d) -= 2 T(q)
//   hbar partial += 2 D-bar(s, d) D(s, d)  (the pair and its mirror)
// Each pair is evaluated by exactly one tile (tiles do not overlap); the
// contributions of a tile land in an LDS region covering q and q + d, written
// out per tile, and a gather forms the padded-grid gradient.  Phase 4 gives
// each thread a run of positions q of the widened tile whose T sums stay in
// its registers; only the q + d terms are read-modify-writes of the region.
#include <cmath>

#include "internal.h"

namespace dsnlm {

namespace {

template <int P, int S_CLASS>
struct DGeo {
    static constexpr int TH = 32, TW = 64, R = 8, L = 4;  // L = 4: one float4 of D-bar per thread
    static constexpr int NT = TH * (TW / L);  // 512
    static constexpr int TWE = TW + 2 * P;
    static constexpr int NITEM1 = TWE * (TH / R);
    static constexpr int GW = 1;  // shifts sharing a register window of the shifted column
    // guide rows ti0-P .. ti0+TH+S+P (+ window slack), column-major, odd stride
    static constexpr int ZC = (TH + S_CLASS + 2 * P + GW - 1) | 1;
    static constexpr int VW0 = ((TWE + 3) / 4) * 4;
    static constexpr int VW = ((VW0 / 4) % 2) ? VW0 : VW0 + 4;
    // D-bar, rows -2P..TH+2P; row stride 4 x odd, for conflict-free float4 writes
    static constexpr int DBH = TH + 4 * P, DBW = TW + 4;
    // phase 4 covers the tile widened by P: rows of (TW + 2P) positions cut
    // into segments of L4, one per thread (the last threads of the block, so
    // that the waves doing phase 1 get fewer); the last segment of a row may
    // run past the widened tile (those positions have G = 0)
    static constexpr int L4 = 7;
    static constexpr int NSEG = (TW + 2 * P + L4 - 1) / L4;
    static constexpr int WWP = NSEG * L4;                           // padded widened width
    static constexpr int NQ = (TH + 2 * P) * NSEG;                  // phase-4 threads
    static constexpr int ZWX = WWP - (TW + 2 * P);                  // extra guide columns
    // LDS layouts for phase 4, whose lane l of a wave works on segment q0 + l:
    // with row strides congruent to WWP mod 64 the first position of segment
    // q sits at bank 7q, so the 64 lanes of a read or write hit 64 banks.
    // The vertical box sums (cols -2P..) use stride WWP itself: the last 2P
    // entries of a row are the first 2P of the next, zero in both (phase 3
    // writes columns 0..TW-1 of D-bar, at 2P..TW+2P-1).
    static constexpr int VBH = TH + 2 * P, VBW = WWP;
    static constexpr int VBN = ((VBH * VBW + 2 * P) + 3) & ~3;      // floats of the box sums
    static constexpr int RWc = WWP + 64;                            // region stride (>= WWP + 2S)
    static_assert(2 * S_CLASS <= 64 && TW + 2 * P <= WWP, "layout");
    static_assert(NQ <= NT, "one phase-4 segment per thread");
    static_assert(NITEM1 <= NT, "one phase-1 item per thread");
};

template <int P, int S_CLASS>
size_t d2_lds_floats(int S) {
    using G = DGeo<P, S_CLASS>;
    const size_t ZWr = G::TW + 2 * (S + P) + G::ZWX;
    size_t n = (ZWr * G::ZC + 3) & ~(size_t)3;
    n += (size_t)G::TH * G::VW;
    n += (size_t)G::DBH * G::DBW + (size_t)G::VBN;
    n += (size_t)(G::TH + 2 * P + S) * G::RWc;
    return n;
}

__device__ __forceinline__ int reflect_d(int k, int n) {
    if (k < 0) k = -k - 1;
    if (k >= n) k = 2 * n - 1 - k;
    k = k < 0 ? 0 : k;
    k = k >= n ? n - 1 : k;
    return k;
}

template <int P, int S_CLASS, bool BATCH>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_d2(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles, int S, HatTable hat,
     int ngrp) {
    using G = DGeo<P, S_CLASS>;
    constexpr int NT = G::NT, TH = G::TH, TW = G::TW, R = G::R, L = G::L;
    constexpr int ZC = G::ZC, VW = G::VW, DBW = G::DBW, VBW = G::VBW, RWc = G::RWc;
    constexpr int NE = R + 2 * P;
    extern __shared__ __align__(16) float lds[];
    const int tid = threadIdx.x;

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
    const int ZH = TH + 2 * P + S, ZWr = TW + 2 * (S + P) + G::ZWX;
    const int RH = TH + 2 * P + S, RWr = TW + 2 * P + 2 * S;
    float* Zs = lds;
    int off = (ZWr * ZC + 3) & ~3;
    float* V = lds + off;
    float* Db = V + TH * VW;
    float* VDb = Db + G::DBH * DBW;
    float* Rg = VDb + G::VBN;

    // ---- staging: guide rows ti0-P .. ti0+TH+S+P, columns tj0-S-P .. (mirrored);
    // D-bar, its box sums and the region start at zero
    for (int idx = tid; idx < ZH * ZWr; idx += NT) {
        const int r = idx / ZWr, q = idx - r * ZWr;
        const int gi = reflect_d(ti0 - P + r, n1);
        const int gj = reflect_d(tj0 - S - P + q, n2);
        Zs[q * ZC + r] = d.z[(size_t)gi * n2 + gj];
    }
    for (int idx = tid; idx < G::DBH * DBW + G::VBN + RH * RWc; idx += NT) Db[idx] = 0.f;
    __syncthreads();

    // ---- phase-1 item: one column strip of R rows of s (reference in registers).
    // Waves 0-3 take the first 64 columns of strips 0-3 (one strip per wave,
    // conflict-free), the next threads the remaining 2P columns of each strip.
    const bool has1 = tid < G::NITEM1;
    int strip = tid >> 6, c1 = tid & 63;
    if constexpr (G::TWE > 64) {
        if (tid >= 256) {
            const int e = has1 ? tid - 256 : 0;
            strip = e / (G::TWE - 64);
            c1 = 64 + e - strip * (G::TWE - 64);
        }
    }
    if (!has1) strip = c1 = 0;
    const int zoff = (c1 + S) * ZC + strip * R;  // Zs column c1 + S is global column tj0 - P + c1
    const int voff = strip * R * VW + c1;
    float ref[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) ref[q] = Zs[zoff + q];

    // ---- the tile's own pixels: factors (omegabar and c scaled by -kappa,
    // B'bar, x), guide values, accumulators
    const int pi = tid % TH;
    const int pj = (tid / TH) * L;
    const int gi_own = ti0 + pi, gj_own = tj0 + pj;
    const float nk = -d.kappa;
    const unsigned long long key = *d.key;
    const int sstar = (int)(~(unsigned)(key & 0xffffffffu));
    const int si = sstar / n2, sj = sstar - si * n2;
    const float mb = *d.mbar;
    const bool fnear = si >= ti0 - S && si < ti0 + TH + S && sj >= tj0 - S && sj < tj0 + TW + S;
    const bool s_in = ti0 + TH <= n1 && tj0 + TW <= n2;
    // partner factors: float4 per pixel, column-major (entry j n1 + i); the
    // buffer starts at the first column the tile's partners can reach and its
    // range check returns zeros past the array (those pairs are masked)
    const int col0 = tj0 - S > 0 ? tj0 - S : 0;
    const float4* img4 = reinterpret_cast<const float4*>(d.aux5) + kAux4Lead;
    const size_t recs = ((size_t)(n2 - col0) * n1 + kAux4Lead + kAux4Trail) * 16;
    // the base and size are uniform: keep them in scalar registers, so each
    // partner load is a single buffer instruction
    const unsigned long long rb = reinterpret_cast<unsigned long long>(img4 + (size_t)col0 * n1 - kAux4Lead);
    const unsigned rlo = __builtin_amdgcn_readfirstlane((unsigned)rb);
    const unsigned rhi = __builtin_amdgcn_readfirstlane((unsigned)(rb >> 32));
    const int rn = __builtin_amdgcn_readfirstlane((int)(recs < 0x7ffffff0u ? recs : 0x7ffffff0u));
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<void*>(((unsigned long long)rhi << 32) | rlo), (short)0, rn, 0x00020000);
    float ow[L], oc[L], ob[L], ox[L];
    // byte offset of the partner of output 0 at shift 0; output k adds k n1 16
    const int roff = ((gj_own - col0) * n1 + gi_own + kAux4Lead) * 16;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int gj = gj_own + k;
        const bool in = gi_own < n1 && gj < n2;
        const float4 o = in ? img4[(size_t)gj * n1 + gi_own] : make_float4(0.f, 0.f, 0.f, 0.f);
        ow[k] = nk * o.x;
        oc[k] = nk * o.y;
        ob[k] = o.z;
        ox[k] = o.w;
    }
    // phase-4 role: a segment of L4 positions q of the widened tile (row qr,
    // first column qc, tile coordinates), their guide values and the sums of T
    constexpr int L4 = G::L4;
    const bool has4 = tid >= NT - G::NQ;
    const int q4 = has4 ? tid - (NT - G::NQ) : 0;
    const int qr = q4 / G::NSEG - P;
    const int qc = (q4 - (qr + P) * G::NSEG) * L4 - P;
    // loop-invariant parts of the phase-4 addresses (each shift adds a
    // wave-uniform offset: one addition per pointer instead of a multiply)
    const int vq0 = (qr + P) * VBW + qc + P;
    const int zq0 = (qc + P) * ZC + qr + P;
    const int rq0 = (qr + P) * RWc + qc + P + S;
    float zown[L4], accz[L4];
    float hsum = 0.f;  // sum of D-bar D over the tile's pairs
#pragma unroll
    for (int k = 0; k < L4; ++k) {
        zown[k] = Zs[(qc + k + P + S) * ZC + qr + P];
        accz[k] = 0.f;
    }

    float4 rv[L];
    auto loadr = [&](int dy, int dx) {
        const int o = (dx * n1 + dy) * 16;
        // keep these loads at this point of the schedule: hoisting them into
        // earlier shifts only raises register pressure
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < L; ++k)
            rv[k] = __builtin_bit_cast(
                float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, roff + (o + k * n1 * 16), 0, 0));
        __builtin_amdgcn_sched_barrier(0);
    };

    // phase 2 + D-bar: horizontal sliding box of V gives D, then
    // -kappa a (abar_{s,d} + abar_{s+d,-d}) with r = s + d:
    //   -kappa (omegabar_s + omegabar_r)
    //   - kappa c_s c_r ((B'bar_s - B'bar_r)(x_r - x_s) + f_s + f_r)
    constexpr int NV = ((L + 2 * P + 3) / 4) * 4;
    float lgx = 0.f;  // log2 of the hat's dx factor, set per dx below
    auto math2 = [&](int dy, int dx) {
        float vv[NV];
        const float* vr = V + pi * VW + pj;
#pragma unroll
        for (int q = 0; q < NV / 4; ++q) {
            const float4 t4 = reinterpret_cast<const float4*>(vr)[q];
            vv[4 * q + 0] = t4.x;
            vv[4 * q + 1] = t4.y;
            vv[4 * q + 2] = t4.z;
            vv[4 * q + 3] = t4.w;
        }
        const float lg = hat.lg[dy + S] + lgx;
        float hs = vv[0];
#pragma unroll
        for (int q = 1; q <= 2 * P; ++q) hs += vv[q];
        float Dk[L];
        Dk[0] = hs;
#pragma unroll
        for (int k = 1; k < L; ++k) {
            hs += vv[k + 2 * P] - vv[k - 1];
            Dk[k] = hs;
        }
        float db[L];
        auto abar = [&](int k) {
            const float4 r = rv[k];
            return fmaf(oc[k] * r.y, (ob[k] - r.z) * (r.w - ox[k]), fmaf(nk, r.x, ow[k]));
        };
        const bool inside = s_in && ti0 + TH - 1 + dy < n1 && tj0 + dx >= 0 && tj0 + TW - 1 + dx < n2;
        if (inside && !fnear) {
#pragma unroll
            for (int k = 0; k < L; ++k) db[k] = __builtin_amdgcn_exp2f(lg - d.beta * Dk[k]) * abar(k);
        } else {
            const bool rowok = gi_own < n1 && gi_own + dy < n1;
            const bool rs = gi_own + dy == si, ss = gi_own == si;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                float as = abar(k);
                if (fnear) {  // the f terms live on s* alone
                    const float fr = (rs && gj_own + k + dx == sj) ? mb : 0.f;
                    const float fs = (ss && gj_own + k == sj) ? mb : 0.f;
                    as = fmaf(oc[k] * rv[k].y, fs + fr, as);
                }
                const float a = __builtin_amdgcn_exp2f(lg - d.beta * Dk[k]);
                const bool ok = rowok && gj_own + k < n2 && (unsigned)(gj_own + k + dx) < (unsigned)n2;
                db[k] = ok ? a * as : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < L; ++k) hsum = fmaf(db[k], Dk[k], hsum);
        *reinterpret_cast<float4*>(Db + (pi + 2 * P) * DBW + pj) = make_float4(db[0], db[1], db[2], db[3]);
    };

    // phase 3: vertical box of D-bar for rows -P..TH+P-1 (column strips)
    auto phase3 = [&]() {
        constexpr int R3 = (TH + 2 * P + 7) / 8;
        const int c = tid % TW, s3 = tid / TW;
        const int r0 = s3 * R3 - P;
        const int r1 = (r0 + R3 < TH + P) ? r0 + R3 : TH + P;
        if (r0 < r1) {
            const float* col = Db + c;
            float v = col[(r0 + P) * DBW];
#pragma unroll
            for (int t = 1 - P; t <= P; ++t) v += col[(r0 + t + 2 * P) * DBW];
            VDb[(r0 + P) * VBW + c + 2 * P] = v;
            for (int r = r0 + 1; r < r1; ++r) {
                v += col[(r + P + 2 * P) * DBW] - col[(r - P - 1 + 2 * P) * DBW];
                VDb[(r + P) * VBW + c + 2 * P] = v;
            }
        }
    };

    // phase 4: horizontal box gives G(q); T = (z(q) - z(q+d)) G(q) is kept
    // at q (registers) and subtracted at q + d (region)
    auto phase4 = [&](int dy, int dx) {
        if (has4) {
            // every read before the first write: the writes could alias the
            // reads as far as the compiler knows, and would force reloads
            const float* vr = VDb + vq0;
            const float* zq = Zs + zq0 + ((S + dx) * ZC + dy);
            float* rq = Rg + rq0 + (dy * RWc + dx);
            float vq[L4 + 2 * P], zs[L4], rg[L4];
#pragma unroll
            for (int q = 0; q < L4 + 2 * P; ++q) vq[q] = vr[q];
#pragma unroll
            for (int k = 0; k < L4; ++k) {
                zs[k] = zq[k * ZC];
                rg[k] = rq[k];
            }
            float hs = vq[0];
#pragma unroll
            for (int q = 1; q <= 2 * P; ++q) hs += vq[q];
#pragma unroll
            for (int k = 0; k < L4; ++k) {
                if (k > 0) hs += vq[k + 2 * P] - vq[k - 1];
                const float t = (zown[k] - zs[k]) * hs;
                accz[k] += t;
                rg[k] -= t;
            }
#pragma unroll
            for (int k = 0; k < L4; ++k) rq[k] = rg[k];
        }
    };

    // shifts of the half window: dx outer, dy inner in groups of GW that
    // share a register window of the shifted guide column.  Phase 3 of a
    // shift shares a barrier interval with phase 1 of the next, phase 4 with
    // its phase 2: two barriers per shift.
    constexpr int GW = G::GW;
    constexpr int NW = NE + GW - 1;
    int t = 0, pdy = 0, pdx = 0;
    // a single-image launch may split the dx range over blockIdx.z (a small
    // image would leave CUs idle); each group writes its own region and hbar
    // partial, and the gather adds the groups in order
    const int grp = BATCH ? 0 : (int)blockIdx.z;
    const int dxlo = BATCH ? -S : -S + grp * (2 * S + 1) / ngrp;
    const int dxhi = BATCH ? S + 1 : -S + (grp + 1) * (2 * S + 1) / ngrp;
    for (int dx = -S; dx <= S; ++dx) {
        if (dx < dxlo || dx >= dxhi) continue;  // another group's (uniform)
        // the hat's dx term in a vector register: one addition per shift for
        // log2 Lambda_d (a VALU instruction reads one scalar operand)
        asm("v_mov_b32 %0, %1" : "=v"(lgx) : "s"(hat.lg[dx + S]));
        for (int dy0 = dx > 0 ? 0 : 1; dy0 <= S; dy0 += GW) {
            float win[NW];
            {
                const float* zq = Zs + zoff + dx * ZC + dy0;
#pragma unroll
                for (int q = 0; q < NW; ++q) win[q] = zq[q];
            }
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                const int dy = dy0 + g;
                if (dy <= S) {
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
                    loadr(dy, dx);  // in flight over phase 3, the barrier and phase 4
                    // phase 3 is a chain of LDS round trips on the block's
                    // path to the barrier: raised issue priority lets each
                    // step go as soon as its rows arrive (-1% on the batch;
                    // the same for phase 1, or for phases 4 and 2, gains less)
                    __builtin_amdgcn_s_setprio(1);
                    if (t > 0) phase3();
                    __builtin_amdgcn_s_setprio(0);
                    __syncthreads();
                    if (t > 0) phase4(pdy, pdx);
                    math2(dy, dx);
                    __syncthreads();
                    pdy = dy;
                    pdx = dx;
                    ++t;
                }
            }
        }
    }
    if (t > 0) {  // drain the last shift
        phase3();
        __syncthreads();
        phase4(pdy, pdx);
    }
    __syncthreads();  // every scatter is in the region
    // the T sums at q join the region (each position has one owner)
    if (has4) {
#pragma unroll
        for (int k = 0; k < L4; ++k) Rg[(qr + P) * RWc + qc + k + P + S] += accz[k];
    }
    __syncthreads();
    const int ntx = (n2 + TW - 1) / TW;
    const int lt = ((ti0 / TH) * ntx + tj0 / TW) * ngrp + grp;  // (tile, group)
    float* part = d.dpart + (size_t)lt * RH * RWr;
    for (int idx = tid; idx < RH * RWr; idx += NT) {
        const int r = idx / RWr, q = idx - r * RWr;
        part[idx] = Rg[r * RWc + q];
    }
    // block partial of sum D-bar D over the half window, doubled for the
    // mirrored pairs: fixed-order LDS tree (V is free after the barriers)
    float* red = V;
    red[tid] = 2.f * hsum;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) d.hpart[lt] = red[0];
}

// Gather: every padded-grid pixel q sums, in a fixed order, the partial
// regions of the tiles whose widened region covers it; gz(q) = 2 x the sum.
// map[b] = (image, block of 256 padded-grid pixels).
template <bool BATCH>
__global__ void __launch_bounds__(256)
k_d2_gather(ImgDesc one, const ImgDesc* __restrict__ batch, const int2* __restrict__ map, int S, int P,
            int ngrp) {
    constexpr int TH = 32, TW = 64;
    ImgDesc d;
    int e;
    if constexpr (BATCH) {
        const int2 mb = map[blockIdx.x];
        d = batch[mb.x];
        e = mb.y * 256 + threadIdx.x;
    } else {
        d = one;
        e = blockIdx.x * 256 + threadIdx.x;
    }
    const int n1 = d.n1, n2 = d.n2, W2 = n2 + 2 * P;
    if (e >= (n1 + 2 * P) * W2) return;
    const int qi = e / W2 - P, qj = e % W2 - P;
    const int nty = (n1 + TH - 1) / TH, ntx = (n2 + TW - 1) / TW;
    const int RH = TH + 2 * P + S, RWr = TW + 2 * P + 2 * S;
    const size_t reg = (size_t)RH * RWr;
    auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    int ty0 = fdiv(qi - TH - P - S, TH) + 1, ty1 = fdiv(qi + P, TH);
    int tx0 = fdiv(qj - TW - P - S, TW) + 1, tx1 = fdiv(qj + P + S, TW);
    ty0 = ty0 < 0 ? 0 : ty0;
    tx0 = tx0 < 0 ? 0 : tx0;
    ty1 = ty1 > nty - 1 ? nty - 1 : ty1;
    tx1 = tx1 > ntx - 1 ? ntx - 1 : tx1;
    float acc = 0.f;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            const int r = qi - ty * TH + P, c = qj - tx * TW + P + S;
            for (int g = 0; g < ngrp; ++g)
                acc += d.dpart[((size_t)(ty * ntx + tx) * ngrp + g) * reg + (size_t)r * RWr + c];
        }
    d.gz[e] = 2.f * acc;
}

template <int P, int S_CLASS, bool BATCH>
hipError_t launch_d2_one(int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles,
                         hipStream_t st) {
    using G = DGeo<P, S_CLASS>;
    const size_t lds = d2_lds_floats<P, S_CLASS>(S) * sizeof(float);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_d2<P, S_CLASS, BATCH>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int ngrp = BATCH ? 1 : sweep_d2_groups(one.n1, one.n2, S);
    const dim3 grid = BATCH ? dim3(ntiles)
                            : dim3((one.n2 + G::TW - 1) / G::TW, (one.n1 + G::TH - 1) / G::TH, ngrp);
    hipLaunchKernelGGL((k_d2<P, S_CLASS, BATCH>), grid, dim3(G::NT), lds, st, one, batch, tiles, S, make_hat(S),
                       ngrp);
    return hipGetLastError();
}

template <int P, bool BATCH>
hipError_t d2_s(int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles, hipStream_t st) {
    if (S <= 12) return launch_d2_one<P, 12, BATCH>(S, one, batch, tiles, ntiles, st);
    return launch_d2_one<P, kMaxS, BATCH>(S, one, batch, tiles, ntiles, st);
}

template <bool BATCH>
hipError_t d2_p(int S, int P, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles,
                hipStream_t st) {
    switch (P) {
        case 0: return d2_s<0, BATCH>(S, one, batch, tiles, ntiles, st);
        case 1: return d2_s<1, BATCH>(S, one, batch, tiles, ntiles, st);
        case 2: return d2_s<2, BATCH>(S, one, batch, tiles, ntiles, st);
        case 3: return d2_s<3, BATCH>(S, one, batch, tiles, ntiles, st);
        case 4: return d2_s<4, BATCH>(S, one, batch, tiles, ntiles, st);
        case 5: return d2_s<5, BATCH>(S, one, batch, tiles, ntiles, st);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
size_t d2_lds_p(int S) {
    return S <= 12 ? d2_lds_floats<P, 12>(S) : d2_lds_floats<P, kMaxS>(S);
}

}  // namespace

bool sweep_d2_fits(int S, int P) {
    size_t f = 0;
    switch (P) {
        case 0: f = d2_lds_p<0>(S); break;
        case 1: f = d2_lds_p<1>(S); break;
        case 2: f = d2_lds_p<2>(S); break;
        case 3: f = d2_lds_p<3>(S); break;
        case 4: f = d2_lds_p<4>(S); break;
        case 5: f = d2_lds_p<5>(S); break;
        default: return false;
    }
    return S <= kMaxS && f * sizeof(float) <= 160 * 1024;
}

int sweep_d2_groups(int n1, int n2, int S) {
    // up to two blocks per CU on 256 CUs, at most 8 groups, at least one dx each
    const int tiles = ((n1 + 31) / 32) * ((n2 + 63) / 64);
    int g = (512 + tiles - 1) / tiles;
    g = g > 8 ? 8 : g;
    return g < 1 ? 1 : (g > 2 * S + 1 ? 2 * S + 1 : g);
}

size_t sweep_d2_part_floats(int n1, int n2, int S, int P) {
    const size_t tiles = (size_t)((n1 + 31) / 32) * ((n2 + 63) / 64);
    return tiles * sweep_d2_groups(n1, n2, S) * (size_t)(32 + 2 * P + S) * (64 + 2 * P + 2 * S);
}

hipError_t launch_sweep_d2(int S, int P, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles,
                           hipStream_t st) {
    ProfScope prof(DSNLM_K_PASS_D, st);
    if (batch) return d2_p<true>(S, P, one, batch, tiles, ntiles, st);
    return d2_p<false>(S, P, one, batch, tiles, ntiles, st);
}

hipError_t launch_d2_gather(int S, int P, const ImgDesc& one, const ImgDesc* batch, const int2* map, int nblocks,
                            hipStream_t st) {
    ProfScope prof(DSNLM_K_BWD_TAIL, st);
    if (batch) {
        hipLaunchKernelGGL((k_d2_gather<true>), dim3(nblocks), dim3(256), 0, st, one, batch, map, S, P, 1);
    } else {
        const int np = (one.n1 + 2 * P) * (one.n2 + 2 * P);
        hipLaunchKernelGGL((k_d2_gather<false>), dim3((np + 255) / 256), dim3(256), 0, st, one, batch, map, S, P,
                           sweep_d2_groups(one.n1, one.n2, S));
    }
    return hipGetLastError();
}

}  // namespace dsnlm
