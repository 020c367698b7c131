// Brute-force DSG-NLM on gfx950: the comparator of Table 1.
//
// Every (pixel, shift) pair sums its patch distance directly over the N_p^2
// patch offsets (no box sums), and the aggregations of Algorithm 2 run as
// written: one kernel forms omega and c = omega^(-1/2) (first loop), one forms
// delta, B' and the running maximum (second and third loops fused by the same
// identity as the fast path, so the outputs are directly comparable), then the
// common epilogue y = x + B'/m.  One thread per pixel; the guide is read from
// a copy mirrored into an S + P margin so no index is reflected in the loop.
#include <cmath>

#include "internal.h"

namespace dsnlm {

namespace {

__device__ __forceinline__ int reflect_b(int k, int n) {
    if (k < 0) k = -k - 1;
    if (k >= n) k = 2 * n - 1 - k;
    k = k < 0 ? 0 : k;
    k = k >= n ? n - 1 : k;
    return k;
}

__global__ void __launch_bounds__(256) k_brute_pad(ImgDesc d, int m) {
    const int W2 = d.n2 + 2 * m, H2 = d.n1 + 2 * m;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= H2 * W2) return;
    const int i = e / W2 - m, j = e % W2 - m;
    d.zpad[e] = d.z[(size_t)reflect_b(i, d.n1) * d.n2 + reflect_b(j, d.n2)];
}

__device__ __forceinline__ unsigned long long wave_max_b(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// PASS 0: omega and c; PASS 1: delta, B' and the packed (delta, index) max.
template <int PASS>
__global__ void __launch_bounds__(256) k_brute(ImgDesc d, int S, int P, HatTable hat) {
    const int n1 = d.n1, n2 = d.n2, m = S + P, W2 = n2 + 2 * m;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if constexpr (PASS == 0) {
        if (idx == 0) *d.key = 0ull;
    }
    unsigned long long best = 0ull;
    if (idx < n1 * n2) {
        const int i = idx / n2, j = idx - i * n2;
        const float* zs = d.zpad + (size_t)(i + m) * W2 + (j + m);  // patch centre of s
        float acc0 = 0.f, acc1 = 0.f;
        for (int dy = -S; dy <= S; ++dy) {
            if ((unsigned)(i + dy) >= (unsigned)n1) continue;
            for (int dx = -S; dx <= S; ++dx) {
                if ((unsigned)(j + dx) >= (unsigned)n2) continue;
                const float* zr = zs + dy * W2 + dx;
                float D = 0.f;
                for (int ty = -P; ty <= P; ++ty)
                    for (int tx = -P; tx <= P; ++tx) {
                        const float t = zs[ty * W2 + tx] - zr[ty * W2 + tx];
                        D = fmaf(t, t, D);
                    }
                const float a = __builtin_amdgcn_exp2f(hat.lg[dy + S] + hat.lg[dx + S] - d.beta * D);
                const size_t r = (size_t)(i + dy) * n2 + (j + dx);
                if constexpr (PASS == 0) {
                    acc0 += a;
                } else {
                    const float cr = d.c[r];
                    acc0 = fmaf(a, cr, acc0);
                    acc1 = fmaf(a, cr * d.x[r], acc1);
                }
            }
        }
        if constexpr (PASS == 0) {
            d.c[idx] = 1.0f / sqrtf(acc0);
        } else {
            const float cs = d.c[idx], xs = d.x[idx];
            const float dl = cs * acc0;
            d.delta[idx] = dl;
            d.bp[idx] = cs * (acc1 - xs * acc0);
            best = ((unsigned long long)__float_as_uint(dl) << 32) | (unsigned long long)(~(unsigned)idx);
        }
    }
    if constexpr (PASS == 1) {
        best = wave_max_b(best);
        if ((threadIdx.x & 63) == 0 && best != 0ull) atomicMax(d.key, best);
    }
}

}  // namespace

hipError_t launch_brute(const ImgDesc& d, int S, int P, hipStream_t st) {
    const int m = S + P;
    const int npad = (d.n1 + 2 * m) * (d.n2 + 2 * m);
    const int n = d.n1 * d.n2;
    const HatTable hat = make_hat(S);
    ProfScope prof(DSNLM_K_PASS_A, st);
    hipLaunchKernelGGL(k_brute_pad, dim3((npad + 255) / 256), dim3(256), 0, st, d, m);
    hipLaunchKernelGGL(k_brute<0>, dim3((n + 255) / 256), dim3(256), 0, st, d, S, P, hat);
    hipLaunchKernelGGL(k_brute<1>, dim3((n + 255) / 256), dim3(256), 0, st, d, S, P, hat);
    return hipGetLastError();
}

}  // namespace dsnlm
