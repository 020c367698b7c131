// Kernel-variant selection for the window sweeps.
//
// Each sweep has more than one compiled schedule (see k_sweep's PIPE
// parameter).  A table maps (sweep kind, search half-width class, patch
// half-width) to the variant to launch.  dsnlm_tune() fills the table by
// timing every variant on the caller's image size; dsnlm_tune_set() pins a
// variant by hand; DSNLM_TUNE_CACHE names a text file the table is loaded from
// at first use and saved to after tuning.
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>

#include "internal.h"

namespace dsnlm {
namespace {

constexpr int kKinds = 4;       // pass A, pass B (both forms), apply, pass C
constexpr int kSClasses = 2;    // S <= 12, S <= 24
constexpr int kPs = kMaxP + 1;

std::mutex g_mu;
int g_table[kKinds][kSClasses][kPs];
bool g_loaded = false;

int kind_of(int mode) {
    switch (mode) {
        case kPassA: return 0;
        case kPassBApply:
        case kPassBBuild: return 1;
        case kApply: return 2;
        default: return 3;
    }
}

void load_cache_locked() {
    if (g_loaded) return;
    g_loaded = true;
    // default: the half-window sweeps (variant 3), the fastest on gfx950
    // for every kind measured (the full-window grouped schedule, variant 2,
    // serves callers without a partial buffer)
    for (auto& a : g_table)
        for (auto& b : a)
            for (int& c : b) c = kHalfVariant;
    const char* path = std::getenv("DSNLM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    int k, sc, p, v;
    while (std::fscanf(f, "%d %d %d %d", &k, &sc, &p, &v) == 4)
        if (k >= 0 && k < kKinds && sc >= 0 && sc < kSClasses && p >= 0 && p < kPs && v >= 0 && v < kSweepVariants)
            g_table[k][sc][p] = v;
    std::fclose(f);
}

void save_cache_locked() {
    const char* path = std::getenv("DSNLM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (int k = 0; k < kKinds; ++k)
        for (int sc = 0; sc < kSClasses; ++sc)
            for (int p = 0; p < kPs; ++p) std::fprintf(f, "%d %d %d %d\n", k, sc, p, g_table[k][sc][p]);
    std::fclose(f);
}

}  // namespace

int sweep_variant(int mode, int S, int P) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    return g_table[kind_of(mode)][S <= 12 ? 0 : 1][P < 0 || P > kMaxP ? 0 : P];
}

void set_sweep_variant(int kind, int S, int P, int v) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    g_table[kind][S <= 12 ? 0 : 1][P] = v;
}

void save_tuning() {
    std::lock_guard<std::mutex> lk(g_mu);
    save_cache_locked();
}

}  // namespace dsnlm

using namespace dsnlm;

extern "C" {

int dsnlm_tune_set(int kind, int S, int P, int variant) {
    if (kind < 0 || kind >= kKinds) return fail(DSNLM_EINVAL, "dsnlm_tune_set: bad kind");
    if (S < 0 || S > kMaxS || P < 0 || P > kMaxP) return fail(DSNLM_EINVAL, "dsnlm_tune_set: bad S or P");
    if (variant < 0 || variant >= kSweepVariants) return fail(DSNLM_EINVAL, "dsnlm_tune_set: bad variant");
    set_sweep_variant(kind, S, P, variant);
    return DSNLM_OK;
}

int dsnlm_tune_get(int kind, int S, int P, int* variant) {
    if (kind < 0 || kind >= kKinds || !variant) return fail(DSNLM_EINVAL, "dsnlm_tune_get: bad argument");
    if (S < 0 || S > kMaxS || P < 0 || P > kMaxP) return fail(DSNLM_EINVAL, "dsnlm_tune_get: bad S or P");
    const int modes[kKinds] = {kPassA, kPassBApply, kApply, kPassC};
    *variant = sweep_variant(modes[kind], S, P);
    return DSNLM_OK;
}

}  // extern "C"

namespace dsnlm {
int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
int prepare_handle(int n1, int n2, int S, int P, float h, dsnlm_weights** out);
ImgDesc base_desc(const dsnlm_weights* w);
}  // namespace dsnlm

extern "C" int dsnlm_tune(const float* guide, int n1, int n2, int S, int P, float h, int reps, void* stream) {
    if (!guide || reps < 1) return fail(DSNLM_EINVAL, "dsnlm_tune: need a guide and reps >= 1");
    int rc = check_denoiser_args(n1, n2, S, P, h, "dsnlm_tune");
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    dsnlm_weights* w = nullptr;
    rc = prepare_handle(n1, n2, S, P, h, &w);
    if (rc) return rc;
    const size_t n = (size_t)n1 * n2;
    float* scratch = nullptr;  // y and the backward per-pixel pair array
    rc = check_hip(hipMalloc(&scratch, (5 * n + 2 * kFacLead) * sizeof(float)), "dsnlm_tune scratch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) rc = check_hip(hipEventCreate(&e0), "event");
    if (!rc) rc = check_hip(hipEventCreate(&e1), "event");
    if (!rc) rc = check_hip(hipMemcpyAsync(w->guide, guide, n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    ImgDesc d = base_desc(w);
    d.x = w->guide;
    d.y = scratch;
    d.aux_in = scratch + n + 2 * kFacLead;  // timing only: the values are irrelevant
    d.aux_out = scratch + 3 * n + 2 * kFacLead;
    // build once so c, delta and m hold meaningful values
    if (!rc) rc = check_hip(launch_sweep(kPassA, S, P, d, nullptr, nullptr, 0, st), "tune build");
    if (!rc) rc = check_hip(launch_sweep(kPassBApply, S, P, d, nullptr, nullptr, 0, st), "tune build");
    if (!rc) rc = check_hip(hipMemcpyAsync(scratch + n + 2 * kFacLead, w->c, n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    if (!rc) rc = check_hip(hipMemcpyAsync(scratch + 2 * n + 2 * kFacLead, w->c, n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    const int modes[4] = {kPassA, kPassBApply, kApply, kPassC};
    for (int k = 0; k < 4 && !rc; ++k) {
        float best = 1e30f;
        int bestv = 0;
        for (int v = 0; v < kSweepVariants && !rc; ++v) {
            set_sweep_variant(k, S, P, v);
            // pass A rewrites c; time it last among the rebuilds it affects
            rc = check_hip(launch_sweep(modes[k], S, P, d, nullptr, nullptr, 0, st), "tune warm-up");
            if (!rc) rc = check_hip(hipEventRecord(e0, st), "event");
            for (int r = 0; r < reps && !rc; ++r)
                rc = check_hip(launch_sweep(modes[k], S, P, d, nullptr, nullptr, 0, st), "tune launch");
            if (!rc) rc = check_hip(hipEventRecord(e1, st), "event");
            if (!rc) rc = check_hip(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (!rc && ms < best) {
                best = ms;
                bestv = v;
            }
        }
        if (!rc) set_sweep_variant(k, S, P, bestv);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(scratch);
    dsnlm_weights_destroy(w);
    if (!rc) save_tuning();
    return rc;
}
