// Kernel timing: while a profiling window is open, launches of the selected kernel kinds
// are bracketed by HIP events recorded on the stream the kernel runs on. Durations are
// resolved when the window closes. Used by the benchmark to time the dominant kernel in
// its timed region; off by default (no events, no overhead).
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <vector>

#include "hsgd_internal.h"

namespace hsgd {

namespace {

struct Rec {
    int kind;
    hipEvent_t a, b;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;     // created lazily, reused across windows
    size_t used = 0;
    std::vector<Rec> recs;
    int64_t launches[kNumKinds] = {};
    double total_ms[kNumKinds] = {};
    int64_t dropped = 0;
};

Profiler& prof() {
    static Profiler p;
    return p;
}

constexpr size_t kMaxRecs = 1 << 16;

hipEvent_t take_event(Profiler& p) {
    if (p.used == p.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p.pool.push_back(e);
    }
    return p.pool[p.used++];
}

}  // namespace

const char* kind_name(int k) {
    static const char* names[kNumKinds] = {"k_select", "k_scan", "k_compact", "k_render",
                                           "k_grad", "k_update", "k_fill_zero", "k_reduce",
                                           "k_upsample", "k_downsample", "k_convert", "k_plane_sweep"};
    return (k >= 0 && k < kNumKinds) ? names[k] : "";
}

ProfScope::ProfScope(int kind, hipStream_t s) : kind_(kind), s_(s) {
    Profiler& p = prof();
    if (!p.on) return;  // racy read is fine: windows are opened/closed between launches
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on || !((p.mask >> kind) & 1u)) return;
    if (p.recs.size() >= kMaxRecs) {
        ++p.dropped;
        return;
    }
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return;
    if (hipEventRecord(a, s) != hipSuccess) return;
    a_ = a;
    b_ = b;
}

ProfScope::~ProfScope() {
    if (!a_) return;
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (hipEventRecord((hipEvent_t)b_, s_) == hipSuccess)
        p.recs.push_back(Rec{kind_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace hsgd

using namespace hsgd;

extern "C" {

hsgd_status hsgd_profile_begin(uint32_t kind_mask) {
    clear_error();
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (p.on) return fail(HSGD_E_ARG, "hsgd_profile_begin: a window is already open");
    p.recs.clear();
    p.used = 0;
    p.dropped = 0;
    for (int k = 0; k < kNumKinds; ++k) {
        p.launches[k] = 0;
        p.total_ms[k] = 0.0;
    }
    p.mask = kind_mask;
    p.on = true;
    return HSGD_OK;
}

hsgd_status hsgd_profile_end(void) {
    clear_error();
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on) return fail(HSGD_E_ARG, "hsgd_profile_end: no window is open");
    p.on = false;
    for (const Rec& r : p.recs) {
        if (hipEventSynchronize(r.b) != hipSuccess)
            return fail(HSGD_E_HIP, "hsgd_profile_end: event synchronisation failed");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return fail(HSGD_E_HIP, "hsgd_profile_end: elapsed time unavailable");
        p.launches[r.kind] += 1;
        p.total_ms[r.kind] += ms;
    }
    p.recs.clear();
    return HSGD_OK;
}

hsgd_status hsgd_profile_read(int32_t kind, int64_t* launches, double* total_ms) {
    clear_error();
    if (kind < 0 || kind >= kNumKinds || !launches || !total_ms)
        return fail(HSGD_E_ARG, "hsgd_profile_read: bad kind or NULL output");
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    *launches = p.launches[kind];
    *total_ms = p.total_ms[kind];
    return HSGD_OK;
}

const char* hsgd_kernel_name(int32_t kind) { return kind_name(kind); }

}  // extern "C"
