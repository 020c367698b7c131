// Allocation-free form of the single-image DSG-NLM forward, for callers that
// cannot allocate device memory (work under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// The intermediates that dsnlm_forward keeps in a handle -- c, delta, B', the
// packed (m, argmax) key, the half-window partial regions, the mirrored guide
// and the extra shift groups' regions -- live instead in one file-scope device
// array of fixed size.  Each device holds its own copy of the array until the
// process ends; its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels.  The kernels
// are the same as dsnlm_forward's, launched with the same descriptor, so the
// two entry points give identical results whenever the array holds the
// partial regions of dsnlm_forward's shift split; for larger images the split
// is reduced to fit (the sums then differ by the order of FP32 additions).
#include <mutex>
#include <string>

#include "internal.h"

namespace dsnlm {
namespace {

// 12 Mi floats = 48 MiB per device.
constexpr size_t kNoAllocFloats = size_t(12) << 20;

__device__ __align__(256) float scratch[kNoAllocFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_dev_scratch[kMaxDevices];  // device address of `scratch` per device (null until looked up)

size_t up64(size_t f) { return (f + 63) & ~size_t(63); }

// Layout inside the array (floats, each part 256-byte aligned): the key
// (64 floats reserved), c, delta, B', the half-window partial buffer
// (regions + mirrored guide), the extra shift groups' regions.
struct Layout {
    size_t key, c, delta, bp, part, gpart, total;
    int groups;
};

// The shift groups are those of dsnlm_forward for this size, reduced to the
// largest count whose regions still fit in the array.
Layout layout(int n1, int n2, int S, int P) {
    Layout L{};
    const size_t n = (size_t)n1 * n2;
    L.key = 0;
    L.c = 64;
    L.delta = L.c + up64(n);
    L.bp = L.delta + up64(n);
    L.part = L.bp + up64(n);
    L.gpart = L.part + up64(half_part_floats(n1, n2, S, P));
    for (L.groups = half_split_groups(n1, n2, S, P);; --L.groups) {
        L.total = L.gpart + up64(half_group_floats(n1, n2, S, L.groups));
        if (L.groups <= 1 || L.total <= kNoAllocFloats) break;
    }
    return L;
}

// Device address of the current device's array (looked up on first use).
int device_scratch(float** out) {
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "dsnlm_forward_noalloc: hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(DSNLM_EUNSUPPORTED, "dsnlm_forward_noalloc: device index >= 64");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev_scratch[dev]) {
        void* p = nullptr;
        rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "dsnlm_forward_noalloc: hipGetSymbolAddress");
        if (rc) return rc;
        if (!p) return fail(DSNLM_EDEVICE, "dsnlm_forward_noalloc: null scratch address");
        g_dev_scratch[dev] = static_cast<float*>(p);
    }
    *out = g_dev_scratch[dev];
    return DSNLM_OK;
}

}  // namespace

int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
bool overlaps(const void* a, const void* b, size_t bytes);

}  // namespace dsnlm

using namespace dsnlm;

extern "C" {

size_t dsnlm_forward_noalloc_limit(void) { return kNoAllocFloats * sizeof(float); }

size_t dsnlm_forward_noalloc_bytes(int n1, int n2, int S, int P) {
    if (n1 < 1 || n2 < 1 || S < 0 || P < 0 || S > kMaxS || P > kMaxP) return 0;
    return layout(n1, n2, S, P).total * sizeof(float);
}

int dsnlm_forward_noalloc(const float* guide, const float* x, float* y, int n1, int n2, int S, int P,
                          float h, void* stream) {
    if (!guide || !x || !y) return fail(DSNLM_EINVAL, "dsnlm_forward_noalloc: null pointer");
    int rc = check_denoiser_args(n1, n2, S, P, h, "dsnlm_forward_noalloc");
    if (rc) return rc;
    const size_t bytes = (size_t)n1 * n2 * sizeof(float);
    if (overlaps(x, y, bytes) || overlaps(guide, y, bytes))
        return fail(DSNLM_EINVAL, "dsnlm_forward_noalloc: y overlaps x or the guide");
    const Layout L = layout(n1, n2, S, P);
    if (L.total > kNoAllocFloats)
        return fail(DSNLM_EUNSUPPORTED, "dsnlm_forward_noalloc: an image of " + std::to_string(n1) + " x " +
                                            std::to_string(n2) + " at S = " + std::to_string(S) + ", P = " +
                                            std::to_string(P) + " needs " +
                                            std::to_string(L.total * sizeof(float)) +
                                            " bytes of scratch; the fixed scratch holds " +
                                            std::to_string(kNoAllocFloats * sizeof(float)));
    float* base = nullptr;
    rc = device_scratch(&base);
    if (rc) return rc;

    ImgDesc d{};
    d.z = guide;  // read in place: nothing is copied
    d.x = x;
    d.y = y;
    d.key = reinterpret_cast<unsigned long long*>(base + L.key);  // reset by pass A
    d.c = base + L.c;
    d.delta = base + L.delta;
    d.bp = base + L.bp;
    d.part = base + L.part;
    d.zpad = half_zpad(d.part, n1, n2, S, P);
    if (L.groups > 1) {
        d.gpart = base + L.gpart;
        d.groups = L.groups;
    }
    d.n1 = n1;
    d.n2 = n2;
    const double np = 2.0 * P + 1.0;
    const double kappa = 1.0 / (2.0 * np * np * (double)h * (double)h);
    d.kappa = (float)kappa;
    d.beta = (float)(kappa * 1.4426950408889634);
    d.h = h;
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = check_hip(launch_sweep(kPassA, S, P, d, nullptr, nullptr, 0, st), "dsnlm_forward_noalloc: pass A");
    if (!rc) rc = check_hip(launch_sweep(kPassBApply, S, P, d, nullptr, nullptr, 0, st), "dsnlm_forward_noalloc: pass B");
    if (!rc) rc = check_hip(launch_epilogue(d, nullptr, nullptr, 0, S, P, st), "dsnlm_forward_noalloc: epilogue");
    return rc;
}

}  // extern "C"
