// Peak-rate probes used as roofline denominators: FP32 FMA issue rate,
// v_exp_f32 rate, HBM copy bandwidth and LDS read bandwidth, each timed with
// HIP events.
#include "internal.h"

namespace dsnlm {
namespace {

// 16 independent FMA chains per lane; 2 ops counted per FMA.
__global__ void __launch_bounds__(256) k_probe_fma(float* out, int iters, float s) {
    float a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = fmaf(a[k], s, 0.5f);
    }
    float r = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) r += a[k];
    if (r == 12345.678f) out[threadIdx.x] = r;  // keeps the chains alive
}

// 16 independent exp2 chains per lane, x <- 2^(-x) (the negation is a free
// source modifier, so each step is one v_exp_f32; the chain stays in (0, 1]).
__global__ void __launch_bounds__(256) k_probe_exp(float* out, int iters) {
    float a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = 1e-3f * (threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = __builtin_amdgcn_exp2f(-a[k]);
    }
    float r = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) r += a[k];
    if (r == 12345.678f) out[threadIdx.x] = r;
}

// Plain copy, 16 bytes per lane per step, grid-stride.
__global__ void __launch_bounds__(256) k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     size_t n4) {
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// LDS reads: 16 bytes per lane per read at fixed, conflict-free addresses
// (consecutive lanes at consecutive 16-byte slots), 8 reads per step, each
// folded into its own accumulator with one 3-input and one 2-input XOR; a
// compiler-only memory fence per step keeps the reads inside the loop.
__global__ void __launch_bounds__(256) k_probe_lds(unsigned* out, int iters) {
    __shared__ uint4 buf[2048];  // 32 KiB
    for (int i = threadIdx.x; i < 2048; i += 256) buf[i] = make_uint4(i, 3 * i, 5 * i, 7 * i);
    __syncthreads();
    unsigned acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = threadIdx.x + k;
    const uint4* p = buf + threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint4 v = p[k * 256];
            acc[k] = (acc[k] ^ v.x ^ v.y) ^ (v.z ^ v.w);
        }
        __asm__ __volatile__("" ::: "memory");
    }
    unsigned r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= acc[k];
    if (r == 0x12345678u) out[threadIdx.x] = r;  // keeps the reads alive
}

}  // namespace
}  // namespace dsnlm

using namespace dsnlm;

// kind 0: FP32 FMA (FLOP/s, 2 per FMA); 1: v_exp_f32 (exp/s); 2: HBM copy
// (bytes/s, read + write); 3: LDS reads (bytes/s over the chip).
extern "C" int dsnlm_peak_probe(int kind, double* rate, void* stream) {
    if (!rate || kind < 0 || kind > 3) return fail(DSNLM_EINVAL, "dsnlm_peak_probe: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 256;
    const int blocks = ncu * 8;
    float* out = nullptr;
    float4 *a = nullptr, *b = nullptr;
    const size_t bytes = (size_t)1 << 30;  // 1 GiB each way for the copy
    int rc = check_hip(hipMalloc(&out, 256 * sizeof(float)), "probe");
    if (!rc && kind == 2) {
        rc = check_hip(hipMalloc(&a, bytes), "probe copy source");
        if (!rc) rc = check_hip(hipMalloc(&b, bytes), "probe copy destination");
        if (!rc) rc = check_hip(hipMemsetAsync(a, 0, bytes, st), "probe init");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) rc = check_hip(hipEventCreate(&e0), "event");
    if (!rc) rc = check_hip(hipEventCreate(&e1), "event");
    const int iters = 4096, reps = 5;
    double work = 0.0;
    for (int r = 0; r <= reps && !rc; ++r) {
        if (r == 1) rc = check_hip(hipEventRecord(e0, st), "event");  // first run is warm-up
        if (kind == 0) {
            hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, out, iters, 0.999f);
            if (r) work += 2.0 * 16 * iters * (double)blocks * 256;
        } else if (kind == 1) {
            hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(256), 0, st, out, iters);
            if (r) work += 16.0 * iters * (double)blocks * 256;
        } else if (kind == 2) {
            hipLaunchKernelGGL(k_probe_copy, dim3(ncu * 16), dim3(256), 0, st, a, b, bytes / 16);
            if (r) work += 2.0 * bytes;
        } else {
            hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(256), 0, st, reinterpret_cast<unsigned*>(out), iters);
            if (r) work += 16.0 * 8 * iters * (double)blocks * 256;
        }
        if (!rc) rc = check_hip(hipGetLastError(), "probe launch");
    }
    if (!rc) rc = check_hip(hipEventRecord(e1, st), "event");
    if (!rc) rc = check_hip(hipEventSynchronize(e1), "event sync");
    float ms = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    if (!rc) *rate = work / (ms * 1e-3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}
