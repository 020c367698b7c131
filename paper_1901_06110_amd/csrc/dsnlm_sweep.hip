// Window sweeps of the DSG-NLM denoiser on gfx950.
//
// Every pass of Algorithm 2 (Section 3) visits, for each pixel s, every pixel
// r = s + d of its search window and needs the kernel weight
//     a_{s,d} = Lambda_d exp(-||P_s - P_{s+d}||^2 / (2 N_p^2 h^2))     (eqs. NLM, S1)
// The sweep kernel below evaluates a_{s,d} for a tile of pixels and one shift d
// at a time and folds it into per-pixel accumulators; what it accumulates
// depends on the pass (SweepMode):
//   pass A : omega_s = sum_d a                        (first aggregation)
//   pass B : sum_d a c_{s+d} and sum_d a c_{s+d} x_{s+d}  (second and third
//            aggregations fused: delta_s and B'_s = c_s sum a c_r (x_r - x_s))
//   apply  : the same sums with weights built earlier (frozen W)
//   pass C : backward sums (same shape as pass B, other per-pixel inputs)
//
// Patch distances for one shift are box sums of the squared-difference image
// e_d(p) = (z(p) - z(p+d))^2 over the (2P+1)^2 patch (the cost-independent-
// of-patch-size idea the paper takes from Darbon et al.); here they are done
// per tile, separably, with short sliding sums:
//   phase 1: threads own a column strip of R rows of the tile widened by P on
//            each side; they form e_d down the strip and a vertical sliding
//            sum of 2P+1 rows, written to LDS;
//   phase 2: threads own a row segment of L output pixels; a horizontal
//            sliding sum over 2P+1 columns of the phase-1 result gives the
//            patch distance, then a = exp2(log2 Lambda_d - beta D).
// The guide tile with an (S+P) halo and the per-pixel inputs with an S halo
// are staged in LDS once per block; HBM traffic is per pixel, not per shift.
// Sliding sums restart every tile (at most R or L steps), so FP32 rounding
// does not build up across the image.
#include "internal.h"

namespace dsnlm {
namespace {

__device__ __forceinline__ int reflect_clamp(int k, int n) {
    // half-sample symmetric mirror (-1 -> 0, n -> n-1); positions beyond one
    // reflection only ever feed pairs whose weight is masked, so clamp them.
    if (k < 0) k = -k - 1;
    if (k >= n) k = 2 * n - 1 - k;
    k = k < 0 ? 0 : k;
    k = k >= n ? n - 1 : k;
    return k;
}

// Tile geometry.  S_CLASS is the largest search half-width the instance
// serves; it fixes the LDS row strides at compile time so every LDS access in
// the shift loop is a base register plus an immediate offset.
template <int P, int S_CLASS>
struct Geo {
    static constexpr int TH = 32, TW = 64;   // output tile
    static constexpr int R = 8;              // phase-1 strip height
    static constexpr int L = 8;              // phase-2 segment length
    static constexpr int NT = TH * (TW / L);  // threads: 256
    static constexpr int TWE = TW + 2 * P;   // tile widened by the patch
    static constexpr int NITEM1 = TWE * (TH / R);
    static constexpr int ROUNDS1 = (NITEM1 + NT - 1) / NT;
    // guide tile, stored column-major: column stride ZC (odd, so lanes that
    // walk along columns hit distinct banks) and at most ZWmax columns
    // (+ GWIN - 1 rows of slack: the register window of the grouped schedule
    // may read past the last valid row of a column; those values are unused)
    static constexpr int GWIN = 7;
    static constexpr int ZC0 = TH + 2 * (S_CLASS + P) + GWIN - 1;
    static constexpr int ZC = (ZC0 % 2) ? ZC0 : ZC0 + 1;
    static constexpr int ZWmax = TW + 2 * (S_CLASS + P);
    // aux row stride: odd, so lanes walking down rows hit distinct banks
    static constexpr int AW = ((TW + 2 * S_CLASS) % 2) ? (TW + 2 * S_CLASS) : (TW + 2 * S_CLASS + 1);
    // V row stride: 4 * odd, for conflict-free float4 reads down rows
    static constexpr int VW0 = ((TWE + 3) / 4) * 4;
    static constexpr int VW = ((VW0 / 4) % 2) ? VW0 : VW0 + 4;
    static_assert(TH % R == 0 && TW % L == 0 && L % 4 == 0, "tile shape");
};

// per-pixel floats staged in LDS: none for pass A (its partners only mask),
// two otherwise
constexpr int naux(int mode) { return mode == kPassA ? 0 : 2; }

template <int P, int S_CLASS>
size_t lds_floats(int S, int mode) {
    using G = Geo<P, S_CLASS>;
    const size_t ZWr = G::TW + 2 * (S + P);
    const size_t AH = G::TH + 2 * S;
    size_t n = (ZWr * G::ZC + 3) & ~(size_t)3;
    n += (AH * G::AW * naux(mode) + 3) & ~(size_t)3;
    n += (size_t)2 * G::TH * G::VW;
    return n;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

template <int P, int S_CLASS, int MODE, bool BATCH, int PIPE>
__global__ void __launch_bounds__(256)
k_sweep(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles, int S,
        HatTable hat) {
    using G = Geo<P, S_CLASS>;
    constexpr int NT = G::NT, TH = G::TH, TW = G::TW, R = G::R, L = G::L;
    constexpr int ZC = G::ZC, AW = G::AW, VW = G::VW;
    constexpr int NA = naux(MODE);
    constexpr int NE = R + 2 * P;  // phase-1 rows per strip
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
        first = blockIdx.x == 0 && blockIdx.y == 0;
    }
    const int n1 = d.n1, n2 = d.n2;
    const int ZH = TH + 2 * (S + P), ZWr = TW + 2 * (S + P);
    const int AH = TH + 2 * S, AWr = TW + 2 * S;
    float* Zs = lds;
    int off = (ZWr * ZC + 3) & ~3;
    float* Aux = lds + off;
    off += (AH * AW * NA + 3) & ~3;
    float* Vb = lds + off;  // two V buffers

    // ---- stage the guide tile (halo S+P, mirrored) and the per-pixel inputs
    for (int idx = tid; idx < ZH * ZWr; idx += NT) {
        const int r = idx / ZWr, q = idx - r * ZWr;
        const int gi = reflect_clamp(ti0 - S - P + r, n1);
        const int gj = reflect_clamp(tj0 - S - P + q, n2);
        Zs[q * ZC + r] = d.z[(size_t)gi * n2 + gj];
    }
    if constexpr (NA == 2) {
        for (int idx = tid; idx < AH * AWr; idx += NT) {
            const int r = idx / AWr, q = idx - r * AWr;
            const int gi = ti0 - S + r, gj = tj0 - S + q;
            const bool in = (unsigned)gi < (unsigned)n1 && (unsigned)gj < (unsigned)n2;
            float2 v = make_float2(0.f, 0.f);  // zero outside: those pairs drop out
            if (in) {
                const size_t p = (size_t)gi * n2 + gj;
                if constexpr (MODE == kPassC) {
                    // backward: t_r = c_r B'bar_r, w_r = c_r (f_r - B'bar_r x_r)
                    v = reinterpret_cast<const float2*>(d.aux_in)[p];
                } else {
                    const float cc = d.c[p];
                    v.x = cc;
                    v.y = (MODE == kPassBBuild) ? 0.f : cc * d.x[p];
                }
            }
            reinterpret_cast<float2*>(Aux)[r * AW + q] = v;
        }
    }
    if constexpr (MODE == kPassA) {
        if (first && tid == 0) *d.key = 0ull;  // pass B takes the max after this
    }
    __syncthreads();

    // ---- phase-1 items of this thread: reference columns kept in registers
    float ref[G::ROUNDS1][NE];
    int zoff[G::ROUNDS1];  // LDS index of the first reference element
    int voff[G::ROUNDS1];  // LDS index (in V) of the first output
#pragma unroll
    for (int k1 = 0; k1 < G::ROUNDS1; ++k1) {
        int it = tid + k1 * NT;
        it = it < G::NITEM1 ? it : G::NITEM1 - 1;  // idle lanes shadow a valid item
        const int strip = it / G::TWE;
        const int c = it - strip * G::TWE;
        zoff[k1] = (c + S) * ZC + strip * R + S;
        voff[k1] = strip * R * VW + c;
#pragma unroll
        for (int q = 0; q < NE; ++q) ref[k1][q] = Zs[zoff[k1] + q];
    }

    const int pi = tid % TH;             // phase-2 output row in the tile
    const int pj = (tid / TH) * L;       // first phase-2 output column
    float acc0[L], acc1[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        acc0[k] = 0.f;
        acc1[k] = 0.f;
    }
    const float beta = d.beta;

    const int NS = (2 * S + 1) * (2 * S + 1);
    const int aux_base = (pi + S) * AW + pj + S;  // own pixel in the per-pixel tile
    const int gi_own = ti0 + pi;
    const int gj_own = tj0 + pj;

    // phase 1: vertical sliding box sums of e_d = (z(p) - z(p+d))^2 down the
    // column strips, written to V.  The running sum adds the entering square
    // and removes the leaving one with two FMAs.
    auto phase1 = [&](int dy, int dx, float* V) {
        const int sh = dx * ZC + dy;
#pragma unroll
        for (int k1 = 0; k1 < G::ROUNDS1; ++k1) {
            if (tid + k1 * NT < G::NITEM1) {
                const float* zq = Zs + zoff[k1] + sh;
                // all reads first: the V stores below may not be reordered
                // above later reads of the same LDS array
                float tq[NE];
#pragma unroll
                for (int q = 0; q < NE; ++q) tq[q] = ref[k1][q] - zq[q];
                float v = tq[0] * tq[0];
#pragma unroll
                for (int q = 1; q <= 2 * P; ++q) v = fmaf(tq[q], tq[q], v);
                float* vo = V + voff[k1];
                vo[0] = v;
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    v = fmaf(tq[q + 2 * P], tq[q + 2 * P], v);
                    v = fmaf(-tq[q - 1], tq[q - 1], v);
                    vo[q * VW] = v;
                }
            }
        }
    };

    // phase 2 is split so its LDS reads can be issued before the next
    // shift's phase 1: load() fetches V (and the per-pixel inputs), math()
    // forms D by horizontal sliding sums and a = exp2(log2 Lambda - beta D).
    constexpr int NV = ((L + 2 * P + 3) / 4) * 4;
    float vv[NV];
    float2 cv[L];
    auto load2 = [&](int dy, int dx, const float* V) {
        const float* vr = V + pi * VW + pj;
#pragma unroll
        for (int q = 0; q < NV / 4; ++q) {
            const float4 t4 = reinterpret_cast<const float4*>(vr)[q];
            vv[4 * q + 0] = t4.x;
            vv[4 * q + 1] = t4.y;
            vv[4 * q + 2] = t4.z;
            vv[4 * q + 3] = t4.w;
        }
        if constexpr (NA == 2) {
            const float2* ap = reinterpret_cast<const float2*>(Aux) + aux_base + (dy * AW + dx);
#pragma unroll
            for (int k = 0; k < L; ++k) cv[k] = ap[k];
        }
    };
    auto math2 = [&](int dy, int dx) {
        const float lg = hat.lg[dy + S] + hat.lg[dx + S];
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
        if constexpr (MODE == kPassA) {
            // the whole tile keeps its partners inside the image for this shift?
            const bool inside = ti0 + dy >= 0 && ti0 + TH - 1 + dy < n1 && tj0 + dx >= 0 &&
                                tj0 + TW - 1 + dx < n2;
            if (inside) {
#pragma unroll
                for (int k = 0; k < L; ++k) acc0[k] += __builtin_amdgcn_exp2f(lg - beta * Dk[k]);
            } else {
                const bool rowok = (unsigned)(gi_own + dy) < (unsigned)n1;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    const float a = __builtin_amdgcn_exp2f(lg - beta * Dk[k]);
                    const bool ok = rowok && (unsigned)(gj_own + k + dx) < (unsigned)n2;
                    acc0[k] += ok ? a : 0.f;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const float a = __builtin_amdgcn_exp2f(lg - beta * Dk[k]);
                acc0[k] = fmaf(a, cv[k].x, acc0[k]);
                if constexpr (MODE != kPassBBuild) acc1[k] = fmaf(a, cv[k].y, acc1[k]);
            }
        }
    };

    // The shift counters advance incrementally (no integer division).  Both
    // schedules use one barrier per shift thanks to the two V buffers.
    int dy = -S, dx = -S;
    if constexpr (PIPE == 2) {
        // grouped schedule: dx outer, dy inner in groups of GWIN shifts.  The
        // shifted column of a strip slides down one row per dy, so one register
        // window of NE + GWIN - 1 values serves the whole group (static indices,
        // fully unrolled) instead of NE LDS reads per shift.
        constexpr int GW = G::GWIN;
        constexpr int NW = NE + GW - 1;
        int t = 0;
        for (dx = -S; dx <= S; ++dx) {
            for (int dy0 = -S; dy0 <= S; dy0 += GW) {
                float win[G::ROUNDS1][NW];
#pragma unroll
                for (int k1 = 0; k1 < G::ROUNDS1; ++k1) {
                    const float* zq = Zs + zoff[k1] + dx * ZC + dy0;
#pragma unroll
                    for (int q = 0; q < NW; ++q) win[k1][q] = zq[q];
                }
#pragma unroll
                for (int g = 0; g < GW; ++g) {
                    if (dy0 + g <= S) {
                        float* V = Vb + (t & 1) * (TH * VW);
#pragma unroll
                        for (int k1 = 0; k1 < G::ROUNDS1; ++k1) {
                            if (tid + k1 * NT < G::NITEM1) {
                                float tq[NE];
#pragma unroll
                                for (int q = 0; q < NE; ++q) tq[q] = ref[k1][q] - win[k1][g + q];
                                float v = tq[0] * tq[0];
#pragma unroll
                                for (int q = 1; q <= 2 * P; ++q) v = fmaf(tq[q], tq[q], v);
                                float* vo = V + voff[k1];
                                vo[0] = v;
#pragma unroll
                                for (int q = 1; q < R; ++q) {
                                    v = fmaf(tq[q + 2 * P], tq[q + 2 * P], v);
                                    v = fmaf(-tq[q - 1], tq[q - 1], v);
                                    vo[q * VW] = v;
                                }
                            }
                        }
                        __syncthreads();
                        load2(dy0 + g, dx, V);
                        math2(dy0 + g, dx);
                        ++t;
                    }
                }
            }
        }
    } else if constexpr (PIPE == 1) {
        // software pipeline: phase 1 of shift t+1 and phase 2 of shift t share
        // one barrier interval (they touch different V buffers)
        phase1(dy, dx, Vb);
        __syncthreads();
        for (int t = 0; t < NS; ++t) {
            int ndx = dx + 1, ndy = dy;
            if (ndx > S) {
                ndx = -S;
                ++ndy;
            }
            load2(dy, dx, Vb + (t & 1) * (TH * VW));
            if (t + 1 < NS) phase1(ndy, ndx, Vb + ((t + 1) & 1) * (TH * VW));
            math2(dy, dx);
            __syncthreads();
            dy = ndy;
            dx = ndx;
        }
    } else {
        for (int t = 0; t < NS; ++t) {
            float* V = Vb + (t & 1) * (TH * VW);
            phase1(dy, dx, V);
            __syncthreads();
            load2(dy, dx, V);
            math2(dy, dx);
            if (++dx > S) {
                dx = -S;
                ++dy;
            }
        }
    }

    // ---- per-pixel epilogue of the pass
    const int gi = ti0 + pi;
    unsigned long long best = 0ull;
    if (gi < n1) {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int gj = tj0 + pj + k;
            if (gj < n2) {
                const size_t p = (size_t)gi * n2 + gj;
                if constexpr (MODE == kPassA) {
                    d.c[p] = 1.0f / sqrtf(acc0[k]);
                } else if constexpr (MODE == kPassC) {
                    // acc0 = sum a t_r, acc1 = sum a w_r
                    reinterpret_cast<float2*>(d.aux_out)[p] = make_float2(acc0[k], acc1[k]);
                } else {
                    const float cs = reinterpret_cast<const float2*>(Aux)[(pi + S) * AW + pj + k + S].x;
                    if constexpr (MODE == kPassBApply || MODE == kApply) {
                        const float xs = d.x[p];
                        d.bp[p] = cs * (acc1[k] - xs * acc0[k]);
                    }
                    if constexpr (MODE == kPassBApply || MODE == kPassBBuild) {
                        const float dl = cs * acc0[k];
                        d.delta[p] = dl;
                        const unsigned long long kk =
                            ((unsigned long long)__float_as_uint(dl) << 32) |
                            (unsigned long long)(~(unsigned)p);
                        best = kk > best ? kk : best;
                    }
                }
            }
        }
    }
    if constexpr (MODE == kPassBApply || MODE == kPassBBuild) {
        best = wave_max_u64(best);
        if ((tid & 63) == 0 && best != 0ull) atomicMax(d.key, best);
    }
}

// y = x + B'/m over one tile (the remainder of Algorithm 2's third loop).
template <int TH, int TW, bool BATCH>
__global__ void __launch_bounds__(256)
k_epilogue(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles) {
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
    const float m = __uint_as_float((unsigned)(*d.key >> 32));
    // a single-image launch splits the tile's rows over gridDim.z blocks
    const int rows = TH / (int)gridDim.z;
    ti0 += (int)blockIdx.z * rows;
    for (int idx = threadIdx.x; idx < rows * TW; idx += 256) {
        const int gi = ti0 + idx / TW, gj = tj0 + idx % TW;
        if (gi < d.n1 && gj < d.n2) {
            const size_t p = (size_t)gi * d.n2 + gj;
            d.y[p] = d.x[p] + d.bp[p] / m;
        }
    }
}

constexpr int kSmallS = 12;  // S <= 12 uses the compact-stride instances

template <int P, int S_CLASS, int MODE, bool BATCH, int PIPE>
hipError_t ensure_attr() {
    static bool attr_set = false;
    if (!attr_set) {
        auto kern = k_sweep<P, S_CLASS, MODE, BATCH, PIPE>;
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    return hipSuccess;
}

template <int P, int S_CLASS, int MODE, bool BATCH, int PIPE>
hipError_t launch_var(int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                      int ntiles, hipStream_t st) {
    using G = Geo<P, S_CLASS>;
    const size_t lds = lds_floats<P, S_CLASS>(S, MODE) * sizeof(float);
    hipError_t e = ensure_attr<P, S_CLASS, MODE, BATCH, PIPE>();
    if (e != hipSuccess) return e;
    dim3 grid = BATCH ? dim3(ntiles) : dim3((one.n2 + G::TW - 1) / G::TW, (one.n1 + G::TH - 1) / G::TH);
    HatTable hat = make_hat(S);
    hipLaunchKernelGGL((k_sweep<P, S_CLASS, MODE, BATCH, PIPE>), grid, dim3(G::NT), lds, st, one,
                       batch, tiles, S, hat);
    return hipGetLastError();
}

template <int P, int S_CLASS, int MODE, bool BATCH>
hipError_t launch_one(int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                      int ntiles, hipStream_t st) {
    switch (sweep_variant(MODE, S, P)) {
        case 0: return launch_var<P, S_CLASS, MODE, BATCH, 0>(S, one, batch, tiles, ntiles, st);
        case 1: return launch_var<P, S_CLASS, MODE, BATCH, 1>(S, one, batch, tiles, ntiles, st);
        default: return launch_var<P, S_CLASS, MODE, BATCH, 2>(S, one, batch, tiles, ntiles, st);
    }
}

template <int P, int S_CLASS, bool BATCH>
hipError_t dispatch_mode(int mode, int S, const ImgDesc& one, const ImgDesc* batch,
                         const TileRef* tiles, int ntiles, hipStream_t st) {
    switch (mode) {
        case kPassA: return launch_one<P, S_CLASS, kPassA, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassBApply: return launch_one<P, S_CLASS, kPassBApply, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassC: return launch_one<P, S_CLASS, kPassC, BATCH>(S, one, batch, tiles, ntiles, st);
        default: break;
    }
    if constexpr (!BATCH) {
        switch (mode) {
            case kPassBBuild: return launch_one<P, S_CLASS, kPassBBuild, false>(S, one, batch, tiles, ntiles, st);
            case kApply: return launch_one<P, S_CLASS, kApply, false>(S, one, batch, tiles, ntiles, st);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <int P, bool BATCH>
hipError_t dispatch_s(int mode, int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                      int ntiles, hipStream_t st) {
    if (S <= kSmallS) return dispatch_mode<P, kSmallS, BATCH>(mode, S, one, batch, tiles, ntiles, st);
    return dispatch_mode<P, kMaxS, BATCH>(mode, S, one, batch, tiles, ntiles, st);
}

template <bool BATCH>
hipError_t dispatch_p(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch,
                      const TileRef* tiles, int ntiles, hipStream_t st) {
    switch (P) {
        case 0: return dispatch_s<0, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 1: return dispatch_s<1, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 2: return dispatch_s<2, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 3: return dispatch_s<3, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 4: return dispatch_s<4, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 5: return dispatch_s<5, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        default: return hipErrorInvalidValue;
    }
}

template <int P, int S_CLASS, int PIPE>
hipError_t prepare_var() {
    hipError_t e = ensure_attr<P, S_CLASS, kPassA, false, PIPE>();
    if (e == hipSuccess) e = ensure_attr<P, S_CLASS, kPassBApply, false, PIPE>();
    if (e == hipSuccess) e = ensure_attr<P, S_CLASS, kPassBBuild, false, PIPE>();
    if (e == hipSuccess) e = ensure_attr<P, S_CLASS, kApply, false, PIPE>();
    if (e == hipSuccess) e = ensure_attr<P, S_CLASS, kPassC, false, PIPE>();
    return e;
}

template <int P, int S_CLASS>
hipError_t prepare_all() {
    hipError_t e = prepare_var<P, S_CLASS, 0>();
    if (e == hipSuccess) e = prepare_var<P, S_CLASS, 1>();
    if (e == hipSuccess) e = prepare_var<P, S_CLASS, 2>();
    return e;
}

template <int P>
hipError_t prepare_p(int S) {
    return S <= kSmallS ? prepare_all<P, kSmallS>() : prepare_all<P, kMaxS>();
}

}  // namespace

HatTable make_hat(int S) {
    HatTable t{};
    for (int k = -S; k <= S; ++k) {
        const double v = 1.0 - std::abs(k) / (double)(S + 1);
        t.lg[k + S] = (float)std::log2(v);
    }
    return t;
}

hipError_t prepare_sweeps(int S, int P) {
    hipError_t e = prepare_half(S, P);
    if (e != hipSuccess) return e;
    switch (P) {
        case 0: return prepare_p<0>(S);
        case 1: return prepare_p<1>(S);
        case 2: return prepare_p<2>(S);
        case 3: return prepare_p<3>(S);
        case 4: return prepare_p<4>(S);
        case 5: return prepare_p<5>(S);
        default: return hipErrorInvalidValue;
    }
}

TileCfg sweep_tile_cfg(int P, int mode) {
    (void)P;
    (void)mode;
    return TileCfg{32, 64, 256};
}

size_t sweep_lds_bytes(int S, int P, int mode) {
    // upper bound over the instances (S_CLASS = 24 for S > 12)
    const int SC = S <= kSmallS ? kSmallS : kMaxS;
    const int TH = 32, TW = 64;
    const size_t ZC = TH + 2 * (SC + P) + 8, AW = TW + 2 * SC + 1, VW = TW + 2 * P + 8;
    size_t n = (TW + 2 * (S + P)) * ZC + (TH + 2 * S) * AW * (mode == kPassA ? 0 : 2) + 2 * TH * VW + 8;
    return n * sizeof(float);
}

hipError_t launch_sweep(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch,
                        const TileRef* tiles, int ntiles, hipStream_t st) {
    const int kind = mode == kPassA ? DSNLM_K_PASS_A
                     : (mode == kPassBApply || mode == kPassBBuild) ? DSNLM_K_PASS_B
                     : mode == kApply ? DSNLM_K_APPLY
                                      : DSNLM_K_PASS_C;
    if (sweep_takes_half(mode, S, P, one) && !(batch && P > kMaxP))
        return launch_half(mode, S, P, one, batch, tiles, ntiles, st);  // times its kernels itself
    if (P > kMaxP) return batch ? hipErrorInvalidValue : launch_wide(mode, S, P, one, st);
    ProfScope prof(kind, st);
    if (batch) return dispatch_p<true>(mode, S, P, one, batch, tiles, ntiles, st);
    return dispatch_p<false>(mode, S, P, one, batch, tiles, ntiles, st);
}

bool sweep_takes_half(int mode, int S, int P, const ImgDesc& one) {
    // wide patches (5 < P <= 15) have the half-window forward sweeps only
    const bool wide_ok = mode == kPassA || mode == kPassBApply || mode == kPassBBuild || mode == kApply;
    return (P <= kMaxP || (P <= kMaxPWide && wide_ok)) && one.part && half_mode_ok(mode) &&
           sweep_variant(mode, S, P) == kHalfVariant && half_lds_fits(S, P, mode);
}

hipError_t launch_epilogue(const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                           int ntiles, int S, int P, hipStream_t st) {
    (void)S;
    (void)P;
    constexpr int TH = 32, TW = 64;
    ProfScope prof(DSNLM_K_EPILOGUE, st);
    if (batch) {
        hipLaunchKernelGGL((k_epilogue<TH, TW, true>), dim3(ntiles), dim3(256), 0, st, one, batch,
                           tiles);
    } else {
        dim3 grid((one.n2 + TW - 1) / TW, (one.n1 + TH - 1) / TH, kGatherSplit);
        hipLaunchKernelGGL((k_epilogue<TH, TW, false>), grid, dim3(256), 0, st, one, batch, tiles);
    }
    return hipGetLastError();
}

}  // namespace dsnlm
