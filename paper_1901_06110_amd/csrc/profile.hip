// Optional per-kernel event timing (dsnlm_profile_* in include/dsnlm.h).
#include <mutex>
#include <vector>

#include "internal.h"

namespace dsnlm {
namespace {

struct Pending {
    int kind;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
double g_ms[DSNLM_K_COUNT];
int g_count[DSNLM_K_COUNT];

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return true;
    return cs != hipStreamCaptureStatusNone;
}

// Fold finished pairs into the totals (caller holds the lock).
void drain(bool wait) {
    std::vector<Pending> keep;
    for (auto& p : g_pending) {
        if (wait) (void)hipEventSynchronize(p.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_ms[p.kind] += ms;
            g_count[p.kind] += 1;
            g_pool.push_back(p.a);
            g_pool.push_back(p.b);
        } else {
            keep.push_back(p);
        }
    }
    g_pending.swap(keep);
}

}  // namespace

ProfScope::ProfScope(int kind, hipStream_t st) : kind_(kind), st_(st), ev_(nullptr) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || capturing(st)) return;
    hipEvent_t a = take_event();
    if (!a) return;
    if (hipEventRecord(a, st) != hipSuccess) {
        g_pool.push_back(a);
        return;
    }
    ev_ = a;
}

ProfScope::~ProfScope() {
    if (!ev_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (!b || hipEventRecord(b, st_) != hipSuccess) {
        g_pool.push_back(ev_);
        if (b) g_pool.push_back(b);
        return;
    }
    g_pending.push_back(Pending{kind_, ev_, b});
    if (g_pending.size() > 4096) drain(true);
}

}  // namespace dsnlm

using namespace dsnlm;

extern "C" {

int dsnlm_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return DSNLM_OK;
}

int dsnlm_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain(true);
    for (int k = 0; k < DSNLM_K_COUNT; ++k) {
        g_ms[k] = 0.0;
        g_count[k] = 0;
    }
    return DSNLM_OK;
}

int dsnlm_profile_query(int kind, double* total_ms, int* launches) {
    if (kind < 0 || kind >= DSNLM_K_COUNT) return fail(DSNLM_EINVAL, "dsnlm_profile_query: bad kind");
    std::lock_guard<std::mutex> lk(g_mu);
    drain(true);
    if (total_ms) *total_ms = g_ms[kind];
    if (launches) *launches = g_count[kind];
    return DSNLM_OK;
}

}  // extern "C"
