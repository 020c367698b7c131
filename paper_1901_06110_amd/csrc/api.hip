// Host side of the C ABI declared in include/dsnlm.h: argument validation,
// handle lifetime, error strings, and the launch sequences of the denoiser.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.h"

namespace dsnlm {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return DSNLM_OK;
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? DSNLM_ENOMEM : DSNLM_EDEVICE;
}

// Validate the denoiser arguments shared by every build/apply entry point
// (pmax: the largest patch half-width the entry point serves).
int check_denoiser_args_p(int n1, int n2, int S, int P, float h, const char* who, int pmax) {
    std::string w(who);
    if (n1 < 1 || n2 < 1) return fail(DSNLM_EINVAL, w + ": image must be at least 1x1");
    if (S < 0 || P < 0) return fail(DSNLM_EINVAL, w + ": S and P must be >= 0");
    if (P >= n1 || P >= n2) return fail(DSNLM_EINVAL, w + ": P must be < min(n1, n2)");
    if (!std::isfinite(h) || !(h > 0.f)) return fail(DSNLM_EINVAL, w + ": h must be finite and > 0");
    if (S > kMaxS || P > pmax)
        return fail(DSNLM_EUNSUPPORTED, w + ": this entry point supports S <= 24 and P <= " + std::to_string(pmax));
    const long long m = (long long)S + P;
    if ((long long)n1 * n2 > kMaxPixels || ((long long)n1 + 2 * m) * ((long long)n2 + 2 * m) > kMaxPixels)
        return fail(DSNLM_EUNSUPPORTED,
                    w + ": the image, or the image padded by S + P on each side, exceeds 2^28 pixels");
    return DSNLM_OK;
}

int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who) {
    return check_denoiser_args_p(n1, n2, S, P, h, who, kMaxP);
}

bool overlaps(const void* a, const void* b, size_t bytes) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bytes && pb < pa + bytes;
}

ImgDesc base_desc(const dsnlm_weights* w) {
    ImgDesc d{};
    d.z = w->guide;
    d.c = w->c;
    d.delta = w->delta;
    d.bp = w->bp;
    d.key = w->key;
    d.part = w->part;
    d.zpad = w->part ? half_zpad(w->part, w->n1, w->n2, w->S, w->P) : nullptr;
    // a small image splits each tile's dx range over several blocks
    const int groups = half_split_groups(w->n1, w->n2, w->S, w->P);
    if (groups > 1 && w->gpart && w->gpart_cap >= half_group_floats(w->n1, w->n2, w->S, groups)) {
        d.gpart = w->gpart;
        d.groups = groups;
    }
    d.n1 = w->n1;
    d.n2 = w->n2;
    // builds that run on the half-window path store pass B's sum of a c for
    // the apply, which then need not form it again (it is fixed with the
    // weights); both build modes must take that path for the apply to rely on it
    if (sweep_takes_half(kPassBApply, w->S, w->P, d) && sweep_takes_half(kPassBBuild, w->S, w->P, d)) d.s0 = w->s0;
    const double np = 2.0 * w->P + 1.0;
    const double kappa = 1.0 / (2.0 * np * np * (double)w->h * (double)w->h);
    d.kappa = (float)kappa;
    d.beta = (float)(kappa * 1.4426950408889634);  // log2(e) * kappa
    d.h = w->h;
    return d;
}

// Create or re-use a handle for an n1 x n2 image.
int prepare_handle(int n1, int n2, int S, int P, float h, dsnlm_weights** out) {
    dsnlm_weights* w = *out;
    if (w && (w->n1 != n1 || w->n2 != n2))
        return fail(DSNLM_EINVAL, "handle was built for a different image size");
    if (!w) {
        w = new (std::nothrow) dsnlm_weights{};
        if (!w) return fail(DSNLM_ENOMEM, "host allocation failed");
        w->n1 = n1;
        w->n2 = n2;
        (void)hipGetDevice(&w->device);
        const size_t n = (size_t)n1 * n2;
        hipError_t e = hipMalloc(&w->guide, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&w->c, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&w->delta, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&w->s0, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&w->bp, n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&w->key, sizeof(unsigned long long));
        if (e != hipSuccess) {
            dsnlm_weights_destroy(w);
            return check_hip(e, "hipMalloc");
        }
        *out = w;
    }
    const size_t need = half_part_floats(n1, n2, S, P);
    if (w->part_cap < need) {
        (void)hipFree(w->part);
        w->part = nullptr;
        w->part_cap = 0;
        int rc = check_hip(hipMalloc(&w->part, need * sizeof(float)), "hipMalloc partial buffer");
        if (rc) return rc;
        w->part_cap = need;
    }
    const size_t gneed = half_group_floats(n1, n2, S, half_split_groups(n1, n2, S, P));
    if (w->gpart_cap < gneed) {
        (void)hipFree(w->gpart);
        w->gpart = nullptr;
        w->gpart_cap = 0;
        int rc = check_hip(hipMalloc(&w->gpart, gneed * sizeof(float)), "hipMalloc group regions");
        if (rc) return rc;
        w->gpart_cap = gneed;
    }
    w->S = S;
    w->P = P;
    w->h = h;
    w->applied = false;
    return DSNLM_OK;
}

}  // namespace dsnlm

using namespace dsnlm;

extern "C" {

const char* dsnlm_last_error(void) { return g_err.c_str(); }

const char* dsnlm_version(void) { return "dsnlm-gfx950 0.1"; }

void dsnlm_weights_destroy(dsnlm_weights* w) {
    if (!w) return;
    (void)hipFree(w->guide);
    (void)hipFree(w->c);
    (void)hipFree(w->delta);
    (void)hipFree(w->s0);
    (void)hipFree(w->bp);
    (void)hipFree(w->key);
    (void)hipFree(w->scratch);
    (void)hipFree(w->bscratch);
    (void)hipFree(w->part);
    (void)hipFree(w->gpart);
    delete w;
}

int dsnlm_build_weights(const float* guide, int n1, int n2, int S, int P, float h, void* stream,
                        dsnlm_weights** out) {
    if (!guide || !out) return fail(DSNLM_EINVAL, "dsnlm_build_weights: null pointer");
    int rc = check_denoiser_args_p(n1, n2, S, P, h, "dsnlm_build_weights", kMaxPWide);
    if (rc) return rc;
    rc = prepare_handle(n1, n2, S, P, h, out);
    if (rc) return rc;
    dsnlm_weights* w = *out;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)n1 * n2 * sizeof(float);
    rc = check_hip(hipMemcpyAsync(w->guide, guide, bytes, hipMemcpyDeviceToDevice, st), "copy guide");
    if (rc) return rc;
    ImgDesc d = base_desc(w);
    rc = check_hip(launch_sweep(kPassA, S, P, d, nullptr, nullptr, 0, st), "pass A");
    if (rc) return rc;
    return check_hip(launch_sweep(kPassBBuild, S, P, d, nullptr, nullptr, 0, st), "pass B");
}

int dsnlm_apply(const dsnlm_weights* wc, const float* x, float* y, void* stream) {
    if (!wc || !x || !y) return fail(DSNLM_EINVAL, "dsnlm_apply: null pointer");
    dsnlm_weights* w = const_cast<dsnlm_weights*>(wc);
    const size_t bytes = (size_t)w->n1 * w->n2 * sizeof(float);
    if (overlaps(x, y, bytes)) return fail(DSNLM_EINVAL, "dsnlm_apply: x and y overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ImgDesc d = base_desc(w);
    d.x = x;
    d.y = y;
    // on the half-window path the gather writes y = x + B'/m itself (m is known)
    const bool fused = sweep_takes_half(kApply, w->S, w->P, d);
    int rc = check_hip(launch_sweep(kApply, w->S, w->P, d, nullptr, nullptr, 0, st), "apply sweep");
    if (rc) return rc;
    if (!fused) rc = check_hip(launch_epilogue(d, nullptr, nullptr, 0, w->S, w->P, st), "epilogue");
    if (rc) return rc;
    w->applied = true;
    return DSNLM_OK;
}

int dsnlm_nlm(const float* guide, const float* x, float* y, int n1, int n2, int S, int P, float h, void* stream,
              dsnlm_weights** out) {
    if (!guide || !x || !y) return fail(DSNLM_EINVAL, "dsnlm_nlm: null pointer");
    int rc = check_denoiser_args(n1, n2, S, P, h, "dsnlm_nlm");
    if (rc) return rc;
    const size_t bytes = (size_t)n1 * n2 * sizeof(float);
    if (overlaps(x, y, bytes) || overlaps(guide, y, bytes))
        return fail(DSNLM_EINVAL, "dsnlm_nlm: y overlaps x or the guide");
    if (!half_lds_fits(S, P, kNLM)) return fail(DSNLM_EUNSUPPORTED, "dsnlm_nlm: S and P too large");
    dsnlm_weights* local = nullptr;
    dsnlm_weights** hp = out ? out : &local;
    rc = prepare_handle(n1, n2, S, P, h, hp);
    if (rc) return rc;
    dsnlm_weights* w = *hp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = check_hip(hipMemcpyAsync(w->guide, guide, bytes, hipMemcpyDeviceToDevice, st), "copy guide");
    ImgDesc d = base_desc(w);
    d.x = x;
    d.y = y;
    if (!rc) rc = check_hip(launch_half(kNLM, S, P, d, nullptr, nullptr, 0, st), "plain NLM sweep");
    if (local) {
        hipError_t e = hipStreamSynchronize(st);
        dsnlm_weights_destroy(local);
        if (!rc) rc = check_hip(e, "dsnlm_nlm: synchronise");
    }
    return rc;
}

int dsnlm_forward_brute(const float* guide, const float* x, float* y, int n1, int n2, int S, int P, float h,
                        void* stream, dsnlm_weights** out) {
    if (!guide || !x || !y) return fail(DSNLM_EINVAL, "dsnlm_forward_brute: null pointer");
    int rc = check_denoiser_args_p(n1, n2, S, P, h, "dsnlm_forward_brute", kMaxPWide);
    if (rc) return rc;
    const size_t bytes = (size_t)n1 * n2 * sizeof(float);
    if (overlaps(x, y, bytes) || overlaps(guide, y, bytes))
        return fail(DSNLM_EINVAL, "dsnlm_forward_brute: y overlaps x or the guide");
    dsnlm_weights* local = nullptr;
    dsnlm_weights** hp = out ? out : &local;
    rc = prepare_handle(n1, n2, S, P, h, hp);
    if (rc) return rc;
    dsnlm_weights* w = *hp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = check_hip(hipMemcpyAsync(w->guide, guide, bytes, hipMemcpyDeviceToDevice, st), "copy guide");
    ImgDesc d = base_desc(w);
    d.x = x;
    d.y = y;
    if (!rc) rc = check_hip(launch_brute(d, S, P, st), "brute-force sweeps");
    if (!rc) rc = check_hip(launch_epilogue(d, nullptr, nullptr, 0, S, P, st), "epilogue");
    if (!rc) w->applied = true;
    if (local) {
        hipError_t e = hipStreamSynchronize(st);
        dsnlm_weights_destroy(local);
        if (!rc) rc = check_hip(e, "dsnlm_forward_brute: synchronise");
    }
    return rc;
}

int dsnlm_forward(const float* guide, const float* x, float* y, int n1, int n2, int S, int P,
                  float h, void* stream, dsnlm_weights** out) {
    if (!guide || !x || !y) return fail(DSNLM_EINVAL, "dsnlm_forward: null pointer");
    int rc = check_denoiser_args_p(n1, n2, S, P, h, "dsnlm_forward", kMaxPWide);
    if (rc) return rc;
    const size_t bytes = (size_t)n1 * n2 * sizeof(float);
    if (overlaps(x, y, bytes) || overlaps(guide, y, bytes))
        return fail(DSNLM_EINVAL, "dsnlm_forward: y overlaps x or the guide");
    dsnlm_weights* local = nullptr;
    dsnlm_weights** hp = out ? out : &local;
    rc = prepare_handle(n1, n2, S, P, h, hp);
    if (rc) return rc;
    dsnlm_weights* w = *hp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = check_hip(hipMemcpyAsync(w->guide, guide, bytes, hipMemcpyDeviceToDevice, st), "copy guide");
    ImgDesc d = base_desc(w);
    d.x = x;
    d.y = y;
    if (!rc) rc = check_hip(launch_sweep(kPassA, S, P, d, nullptr, nullptr, 0, st), "pass A");
    if (!rc) rc = check_hip(launch_sweep(kPassBApply, S, P, d, nullptr, nullptr, 0, st), "pass B");
    if (!rc) rc = check_hip(launch_epilogue(d, nullptr, nullptr, 0, S, P, st), "epilogue");
    if (!rc) w->applied = true;
    if (local) {
        // the temporary handle's buffers must outlive the queued kernels
        hipError_t e = hipStreamSynchronize(st);
        dsnlm_weights_destroy(local);
        if (!rc) rc = check_hip(e, "dsnlm_forward: synchronise");
    }
    return rc;
}

int dsnlm_weights_scalars(const dsnlm_weights* w, float* m, int* argmax, void* stream) {
    if (!w) return fail(DSNLM_EINVAL, "dsnlm_weights_scalars: null handle");
    unsigned long long key = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = check_hip(hipMemcpyAsync(&key, w->key, sizeof(key), hipMemcpyDeviceToHost, st), "copy key");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "synchronise");
    if (rc) return rc;
    unsigned bits = (unsigned)(key >> 32);
    float mv;
    std::memcpy(&mv, &bits, sizeof(mv));
    if (m) *m = mv;
    if (argmax) *argmax = (int)(~(unsigned)(key & 0xffffffffu));
    return DSNLM_OK;
}

const float* dsnlm_weights_array(const dsnlm_weights* w, int which) {
    if (!w) return nullptr;
    switch (which) {
        case 0: return w->c;
        case 1: return w->delta;
        case 2: return w->guide;
        default: return nullptr;
    }
}

}  // extern "C"
