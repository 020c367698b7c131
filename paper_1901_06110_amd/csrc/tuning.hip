// Autotuning of the window sweeps.
//
// Two tables steer the launches:
//   * the schedule ("variant") of each sweep kind, keyed by (kind, search
//     half-width class, patch half-width): the full-window schedules of
//     k_sweep (plain, software-pipelined, grouped register window) or the
//     half-window sweeps of k_half;
//   * the number of blocks a single-image half-window sweep splits each
//     tile's shifts over (the "shift groups": equal contiguous ranges of the
//     half window, each block with its own partial regions), keyed by (search
//     half-width class, patch half-width, image size class by its number of
//     32 x 64 tiles).  A small image has too few tiles to fill 256 CUs; more
//     groups fill them at the cost of more partial regions to gather.
// dsnlm_tune() fills both by timing the candidates on the caller's image;
// dsnlm_tune_set() / dsnlm_tune_set_groups() pin entries by hand;
// DSNLM_TUNE_CACHE names a text file the tables are loaded from at first use
// and saved to after tuning.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace dsnlm {
namespace {

constexpr int kKinds = 4;       // pass A, pass B (both forms), apply, pass C
constexpr int kSClasses = 2;    // S <= 12, S <= 24
constexpr int kPs = kMaxP + 1;
constexpr int kSizeClasses = 7;  // tiles <= 16, 32, 64, 128, 256, 512, more

std::mutex g_mu;
int g_table[kKinds][kSClasses][kPs];
int g_groups[kSClasses][kPs][kSizeClasses];  // 0: the default rule
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

int size_class(int tiles) {
    int c = 0;
    for (int lim = 16; c < kSizeClasses - 1 && tiles > lim; lim *= 2) ++c;
    return c;
}

int tiles_of(int n1, int n2) { return ((n1 + 31) / 32) * ((n2 + 63) / 64); }

void load_cache_locked() {
    if (g_loaded) return;
    g_loaded = true;
    // default: the half-window sweeps (variant 3), the fastest on gfx950
    // for every kind measured (the full-window grouped schedule, variant 2,
    // serves callers without a partial buffer)
    for (auto& a : g_table)
        for (auto& b : a)
            for (int& c : b) c = kHalfVariant;
    std::memset(g_groups, 0, sizeof(g_groups));
    const char* path = std::getenv("DSNLM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char tag[8];
    int a, b, c, v;
    while (std::fscanf(f, "%7s %d %d %d %d", tag, &a, &b, &c, &v) == 5) {
        if (std::strcmp(tag, "v") == 0 && a >= 0 && a < kKinds && b >= 0 && b < kSClasses && c >= 0 && c < kPs &&
            v >= 0 && v < kSweepVariants)
            g_table[a][b][c] = v;
        if (std::strcmp(tag, "g") == 0 && a >= 0 && a < kSClasses && b >= 0 && b < kPs && c >= 0 &&
            c < kSizeClasses && v >= 0 && v <= kMaxShiftGroups)
            g_groups[a][b][c] = v;
    }
    std::fclose(f);
}

void save_cache_locked() {
    const char* path = std::getenv("DSNLM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (int k = 0; k < kKinds; ++k)
        for (int sc = 0; sc < kSClasses; ++sc)
            for (int p = 0; p < kPs; ++p) std::fprintf(f, "v %d %d %d %d\n", k, sc, p, g_table[k][sc][p]);
    for (int sc = 0; sc < kSClasses; ++sc)
        for (int p = 0; p < kPs; ++p)
            for (int c = 0; c < kSizeClasses; ++c)
                if (g_groups[sc][p][c]) std::fprintf(f, "g %d %d %d %d\n", sc, p, c, g_groups[sc][p][c]);
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

int tuned_shift_groups(int n1, int n2, int S, int P) {
    if (P < 0 || P > kMaxP) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    return g_groups[S <= 12 ? 0 : 1][P][size_class(tiles_of(n1, n2))];
}

void set_shift_groups(int n1, int n2, int S, int P, int groups) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    g_groups[S <= 12 ? 0 : 1][P][size_class(tiles_of(n1, n2))] = groups;
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

int dsnlm_tune_set_groups(int n1, int n2, int S, int P, int groups) {
    if (n1 < 1 || n2 < 1 || S < 0 || S > kMaxS || P < 0 || P > kMaxP)
        return fail(DSNLM_EINVAL, "dsnlm_tune_set_groups: bad size, S or P");
    if (groups < 0 || groups > kMaxShiftGroups)
        return fail(DSNLM_EINVAL, "dsnlm_tune_set_groups: groups must be in 0.." + std::to_string(kMaxShiftGroups));
    set_shift_groups(n1, n2, S, P, groups);
    return DSNLM_OK;
}

int dsnlm_tune_get_groups(int n1, int n2, int S, int P, int* groups) {
    if (!groups || n1 < 1 || n2 < 1 || S < 0 || S > kMaxS || P < 0 || P > kMaxP)
        return fail(DSNLM_EINVAL, "dsnlm_tune_get_groups: bad argument");
    *groups = half_split_groups(n1, n2, S, P);
    return DSNLM_OK;
}

}  // extern "C"

namespace dsnlm {
int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
int prepare_handle(int n1, int n2, int S, int P, float h, dsnlm_weights** out);
ImgDesc base_desc(const dsnlm_weights* w);
}  // namespace dsnlm

namespace {

// Device milliseconds of `reps` runs of the launches in fn (after one
// warm-up run), or a negative value on error (rc set).
template <class F>
float time_launches(F fn, int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int* rc) {
    *rc = fn();
    if (!*rc) *rc = check_hip(hipEventRecord(e0, st), "event");
    for (int r = 0; r < reps && !*rc; ++r) *rc = fn();
    if (!*rc) *rc = check_hip(hipEventRecord(e1, st), "event");
    if (!*rc) *rc = check_hip(hipEventSynchronize(e1), "event sync");
    float ms = -1.f;
    if (!*rc) *rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    return *rc ? -1.f : ms;
}

}  // namespace

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
    auto desc = [&]() {
        ImgDesc d = base_desc(w);
        d.x = w->guide;
        d.y = scratch;
        d.aux_in = scratch + n + 2 * kFacLead;  // timing only: the values are irrelevant
        d.aux_out = scratch + 3 * n + 2 * kFacLead;
        return d;
    };
    // build once so c, delta and m hold meaningful values
    if (!rc) rc = check_hip(launch_sweep(kPassA, S, P, desc(), nullptr, nullptr, 0, st), "tune build");
    if (!rc) rc = check_hip(launch_sweep(kPassBApply, S, P, desc(), nullptr, nullptr, 0, st), "tune build");
    if (!rc) rc = check_hip(hipMemcpyAsync(scratch + n + 2 * kFacLead, w->c, n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    if (!rc) rc = check_hip(hipMemcpyAsync(scratch + 2 * n + 2 * kFacLead, w->c, n * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    // 1. the schedule of every sweep kind
    const int modes[4] = {kPassA, kPassBApply, kApply, kPassC};
    for (int k = 0; k < 4 && !rc; ++k) {
        float best = 1e30f;
        int bestv = 0;
        for (int v = 0; v < kSweepVariants && !rc; ++v) {
            set_sweep_variant(k, S, P, v);
            const ImgDesc d = desc();
            // pass A rewrites c; time it last among the rebuilds it affects
            const float ms = time_launches(
                [&]() { return check_hip(launch_sweep(modes[k], S, P, d, nullptr, nullptr, 0, st), "tune launch"); },
                reps, st, e0, e1, &rc);
            if (!rc && ms < best) {
                best = ms;
                bestv = v;
            }
        }
        if (!rc) set_sweep_variant(k, S, P, bestv);
    }
    // 2. the shift groups of a single-image half-window launch of this size:
    // the forward (pass A, pass B) and a frozen apply, for each candidate
    const int H = 2 * S * (S + 1);
    if (!rc && H > 0 && sweep_takes_half(kPassBApply, S, P, desc())) {
        const int cand[] = {1, 2, 3, 4, 5, 6, 8};
        float best = 1e30f;
        int bestg = 1;
        for (int g : cand) {
            if (rc || g > kMaxShiftGroups || g > H) continue;
            set_shift_groups(n1, n2, S, P, g);
            rc = prepare_handle(n1, n2, S, P, h, &w);  // grows the group regions if needed
            if (rc) break;
            const ImgDesc d = desc();
            const float ms = time_launches(
                [&]() {
                    int r = check_hip(launch_sweep(kPassA, S, P, d, nullptr, nullptr, 0, st), "tune launch");
                    if (!r) r = check_hip(launch_sweep(kPassBApply, S, P, d, nullptr, nullptr, 0, st), "tune launch");
                    if (!r) r = check_hip(launch_sweep(kApply, S, P, d, nullptr, nullptr, 0, st), "tune launch");
                    return r;
                },
                reps, st, e0, e1, &rc);
            if (!rc && ms < best) {
                best = ms;
                bestg = g;
            }
        }
        if (!rc) set_shift_groups(n1, n2, S, P, bestg);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(scratch);
    dsnlm_weights_destroy(w);
    if (!rc) save_tuning();
    return rc;
}
