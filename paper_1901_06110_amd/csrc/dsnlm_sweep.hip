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

template <int P, int TH, int TW, int R, int L>
struct Geo {
    static constexpr int NT = TH * (TW / L);        // threads per block
    static constexpr int TWE = TW + 2 * P;          // tile widened by the patch
    static constexpr int NITEM1 = TWE * (TH / R);   // phase-1 work items
    static constexpr int ROUNDS1 = (NITEM1 + NT - 1) / NT;
    static constexpr int VW = ((TWE + 3) / 4) * 4 + 4;  // padded row of V
    static_assert(TH % R == 0, "strip height must divide the tile height");
    static_assert(TW % L == 0, "segment length must divide the tile width");
    static_assert(L % 4 == 0, "segments are read as float4");
};

constexpr int naux(int mode) { return mode == kPassA ? 1 : 2; }

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

template <int P, int TH, int TW, int R, int L, int MODE, bool BATCH>
__global__ void __launch_bounds__(TH * (TW / L))
k_sweep(ImgDesc one, const ImgDesc* __restrict__ batch, const TileRef* __restrict__ tiles, int S,
        HatTable hat) {
    using G = Geo<P, TH, TW, R, L>;
    constexpr int NT = G::NT;
    constexpr int NA = naux(MODE);
    extern __shared__ __align__(16) float lds[];
    const int tid = threadIdx.x;

    ImgDesc d;
    int ti0, tj0;
    bool first;
    if constexpr (BATCH) {
        const TileRef t = tiles[blockIdx.x];
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
    const int ZH = TH + 2 * (S + P), ZW = TW + 2 * (S + P);
    const int AH = TH + 2 * S, AW = TW + 2 * S;
    float* Zs = lds;
    int off = (ZH * ZW + 3) & ~3;
    float* Aux = lds + off;
    off += (AH * AW * NA + 3) & ~3;
    float* Vb = lds + off;

    // ---- stage the guide tile (halo S+P, mirrored) and the per-pixel inputs
    for (int idx = tid; idx < ZH * ZW; idx += NT) {
        const int r = idx / ZW, q = idx - r * ZW;
        const int gi = reflect_clamp(ti0 - S - P + r, n1);
        const int gj = reflect_clamp(tj0 - S - P + q, n2);
        Zs[idx] = d.z[(size_t)gi * n2 + gj];
    }
    for (int idx = tid; idx < AH * AW; idx += NT) {
        const int r = idx / AW, q = idx - r * AW;
        const int gi = ti0 - S + r, gj = tj0 - S + q;
        const bool in = (unsigned)gi < (unsigned)n1 && (unsigned)gj < (unsigned)n2;
        if constexpr (MODE == kPassA) {
            Aux[idx] = in ? 1.f : 0.f;  // pairs leaving the image get weight 0
        } else {
            float2 v = make_float2(0.f, 0.f);
            if (in) {
                const size_t p = (size_t)gi * n2 + gj;
                if constexpr (MODE == kPassC) {
                    // backward: t_r = c_r B'bar_r, w_r = c_r (f_r - B'bar_r x_r)
                    v.x = d.cbar_aux[2 * p];
                    v.y = d.cbar_aux[2 * p + 1];
                } else {
                    const float cc = d.c[p];
                    v.x = cc;
                    v.y = (MODE == kPassBBuild) ? 0.f : cc * d.x[p];
                }
            }
            reinterpret_cast<float2*>(Aux)[idx] = v;
        }
    }
    if constexpr (MODE == kPassA) {
        if (first && tid == 0) *d.key = 0ull;  // pass B takes the max after this
    }
    __syncthreads();

    const int pi = tid / (TW / L);        // phase-2 output row in the tile
    const int pj = (tid % (TW / L)) * L;  // first phase-2 output column
    float acc0[L], acc1[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        acc0[k] = 0.f;
        acc1[k] = 0.f;
    }
    const float beta = d.beta;

    int buf = 0;
    for (int dy = -S; dy <= S; ++dy) {
        const float lgy = hat.lg[dy + S];
        for (int dx = -S; dx <= S; ++dx) {
            const float lg = lgy + hat.lg[dx + S];
            float* V = Vb + buf * (TH * G::VW);
            // ---- phase 1: vertical sliding box sums of e_d down column strips
#pragma unroll
            for (int k1 = 0; k1 < G::ROUNDS1; ++k1) {
                const int it = tid + k1 * NT;
                if (it < G::NITEM1) {
                    const int strip = it / G::TWE;
                    const int c = it - strip * G::TWE;
                    const int r0 = strip * R;
                    const float* zr = Zs + (r0 + S) * ZW + c + S;
                    const float* zq = zr + dy * ZW + dx;
                    float e[R + 2 * P];
#pragma unroll
                    for (int q = 0; q < R + 2 * P; ++q) {
                        const float t = zr[q * ZW] - zq[q * ZW];
                        e[q] = t * t;
                    }
                    float v = 0.f;
#pragma unroll
                    for (int q = 0; q <= 2 * P; ++q) v += e[q];
                    float* vo = V + r0 * G::VW + c;
                    vo[0] = v;
#pragma unroll
                    for (int q = 1; q < R; ++q) {
                        v += e[q + 2 * P] - e[q - 1];
                        vo[q * G::VW] = v;
                    }
                }
            }
            __syncthreads();
            // ---- phase 2: horizontal sliding sums -> D, weights, accumulate
            const float* vr = V + pi * G::VW + pj;
            float vv[((L + 2 * P + 3) / 4) * 4];
#pragma unroll
            for (int q = 0; q < (L + 2 * P + 3) / 4; ++q) {
                const float4 t4 = reinterpret_cast<const float4*>(vr)[q];
                vv[4 * q + 0] = t4.x;
                vv[4 * q + 1] = t4.y;
                vv[4 * q + 2] = t4.z;
                vv[4 * q + 3] = t4.w;
            }
            float hs = 0.f;
#pragma unroll
            for (int q = 0; q <= 2 * P; ++q) hs += vv[q];
            float Dk[L];
            Dk[0] = hs;
#pragma unroll
            for (int k = 1; k < L; ++k) {
                hs += vv[k + 2 * P] - vv[k - 1];
                Dk[k] = hs;
            }
            const int arow = (pi + dy + S) * AW + pj + dx + S;
            if constexpr (NA == 1) {
                const float* ap = Aux + arow;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    const float a = __builtin_amdgcn_exp2f(lg - beta * Dk[k]);
                    acc0[k] = fmaf(a, ap[k], acc0[k]);
                }
            } else {
                const float2* ap = reinterpret_cast<const float2*>(Aux) + arow;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    const float a = __builtin_amdgcn_exp2f(lg - beta * Dk[k]);
                    const float2 cv = ap[k];
                    acc0[k] = fmaf(a, cv.x, acc0[k]);
                    if constexpr (MODE != kPassBBuild) acc1[k] = fmaf(a, cv.y, acc1[k]);
                }
            }
            buf ^= 1;
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
                    // acc0 = sum a t_r = U_s, acc1 = sum a w_r
                    d.cbar_aux[2 * p] = acc0[k];
                    d.cbar_aux[2 * p + 1] = acc1[k];
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
        const TileRef t = tiles[blockIdx.x];
        d = batch[t.img];
        ti0 = t.ti0;
        tj0 = t.tj0;
    } else {
        d = one;
        ti0 = blockIdx.y * TH;
        tj0 = blockIdx.x * TW;
    }
    const float m = __uint_as_float((unsigned)(*d.key >> 32));
    for (int idx = threadIdx.x; idx < TH * TW; idx += 256) {
        const int gi = ti0 + idx / TW, gj = tj0 + idx % TW;
        if (gi < d.n1 && gj < d.n2) {
            const size_t p = (size_t)gi * d.n2 + gj;
            d.y[p] = d.x[p] + d.bp[p] / m;
        }
    }
}

// Tile shape per patch half-width: TH x TW outputs, strips of R rows,
// segments of L columns (256 threads).
template <int P>
struct Shape {
    static constexpr int TH = 32, TW = 64, R = 8, L = 8;
};

template <int P, int MODE, bool BATCH>
hipError_t launch_one(int S, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                      int ntiles, hipStream_t st) {
    using Sh = Shape<P>;
    using G = Geo<P, Sh::TH, Sh::TW, Sh::R, Sh::L>;
    auto kern = k_sweep<P, Sh::TH, Sh::TW, Sh::R, Sh::L, MODE, BATCH>;
    const size_t lds = sweep_lds_bytes(S, P, MODE);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    dim3 grid;
    if (BATCH) {
        grid = dim3(ntiles);
    } else {
        grid = dim3((one.n2 + Sh::TW - 1) / Sh::TW, (one.n1 + Sh::TH - 1) / Sh::TH);
    }
    HatTable hat = make_hat(S);
    hipLaunchKernelGGL(kern, grid, dim3(G::NT), lds, st, one, batch, tiles, S, hat);
    return hipGetLastError();
}

template <int P, bool BATCH>
hipError_t dispatch_mode(int mode, int S, const ImgDesc& one, const ImgDesc* batch,
                         const TileRef* tiles, int ntiles, hipStream_t st) {
    switch (mode) {
        case kPassA: return launch_one<P, kPassA, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassBApply: return launch_one<P, kPassBApply, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassBBuild: return launch_one<P, kPassBBuild, BATCH>(S, one, batch, tiles, ntiles, st);
        case kApply: return launch_one<P, kApply, BATCH>(S, one, batch, tiles, ntiles, st);
        case kPassC: return launch_one<P, kPassC, BATCH>(S, one, batch, tiles, ntiles, st);
        default: return hipErrorInvalidValue;
    }
}

template <bool BATCH>
hipError_t dispatch_p(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch,
                      const TileRef* tiles, int ntiles, hipStream_t st) {
    switch (P) {
        case 0: return dispatch_mode<0, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 1: return dispatch_mode<1, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 2: return dispatch_mode<2, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 3: return dispatch_mode<3, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 4: return dispatch_mode<4, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        case 5: return dispatch_mode<5, BATCH>(mode, S, one, batch, tiles, ntiles, st);
        default: return hipErrorInvalidValue;
    }
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

TileCfg sweep_tile_cfg(int P, int mode) {
    (void)P;
    (void)mode;
    return TileCfg{32, 64, 256};
}

size_t sweep_lds_bytes(int S, int P, int mode) {
    const int TH = 32, TW = 64;
    const int ZH = TH + 2 * (S + P), ZW = TW + 2 * (S + P);
    const int AH = TH + 2 * S, AW = TW + 2 * S;
    const int VW = ((TW + 2 * P + 3) / 4) * 4 + 4;
    size_t n = ((size_t)ZH * ZW + 3) & ~(size_t)3;
    n += ((size_t)AH * AW * naux(mode) + 3) & ~(size_t)3;
    n += (size_t)2 * TH * VW;
    return n * sizeof(float);
}

hipError_t launch_sweep(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch,
                        const TileRef* tiles, int ntiles, hipStream_t st) {
    const int kind = mode == kPassA ? DSNLM_K_PASS_A
                     : (mode == kPassBApply || mode == kPassBBuild) ? DSNLM_K_PASS_B
                     : mode == kApply ? DSNLM_K_APPLY
                                      : DSNLM_K_PASS_C;
    ProfScope prof(kind, st);
    if (batch) return dispatch_p<true>(mode, S, P, one, batch, tiles, ntiles, st);
    return dispatch_p<false>(mode, S, P, one, batch, tiles, ntiles, st);
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
        dim3 grid((one.n2 + TW - 1) / TW, (one.n1 + TH - 1) / TH);
        hipLaunchKernelGGL((k_epilogue<TH, TW, false>), grid, dim3(256), 0, st, one, batch, tiles);
    }
    return hipGetLastError();
}

}  // namespace dsnlm
