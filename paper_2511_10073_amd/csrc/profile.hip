// Optional per-stage timing with HIP events on the caller's stream.  When
// enabled, every stage records an event pair; ahr_profile_read waits for
// them and accumulates the elapsed times.
#include <mutex>

#include "ahr_internal.hpp"

namespace ahr {

namespace {

struct Pending {
    hipEvent_t a, b;
    int stage;
    double bytes;
};

std::mutex g_mu;
int g_on = 0;       // 0 off, 1 every stage, 2 hop launches only
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
double g_ms[kStageCount] = {};
int64_t g_count[kStageCount] = {};
double g_bytes[kStageCount] = {};

hipEvent_t take_event() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e;
    AHR_HIP(hipEventCreate(&e));
    return e;
}

void drain_locked() {
    for (auto& p : g_pending) {
        AHR_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        AHR_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        g_ms[p.stage] += ms;
        g_count[p.stage] += 1;
        g_bytes[p.stage] += p.bytes;
        g_free.push_back(p.a);
        g_free.push_back(p.b);
    }
    g_pending.clear();
}

}  // namespace

thread_local bool t_capture = false;

bool profiling() { return g_on != 0 && !t_capture; }

void set_capture(bool on) { t_capture = on; }

bool prof_kernel_events(Stage st, hipEvent_t* start, hipEvent_t* stop) {
    *start = *stop = nullptr;
    if (!g_on || t_capture || (g_on == 2 && st != kStageHop)) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    *start = take_event();
    *stop = take_event();
    return true;
}

void prof_kernel_done(Stage st, hipEvent_t start, hipEvent_t stop, double bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back(Pending{start, stop, st, bytes});
    if (g_pending.size() > 4096) drain_locked();
}

ProfScope::ProfScope(Stage st, hipStream_t s, double bytes) : stage_(st), s_(s), bytes_(bytes) {
    if (!g_on || t_capture || (g_on == 2 && st != kStageHop)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = take_event();
    AHR_HIP(hipEventRecord(static_cast<hipEvent_t>(a_), s));
    live_ = true;
}

ProfScope::~ProfScope() {
    if (!live_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    try {
        hipEvent_t b = take_event();
        if (hipEventRecord(b, s_) != hipSuccess) return;
        g_pending.push_back(Pending{static_cast<hipEvent_t>(a_), b, stage_, bytes_});
        if (g_pending.size() > 4096) drain_locked();
    } catch (...) {
    }
}

}  // namespace ahr

extern "C" {

ahr_status ahr_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(ahr::g_mu);
    if (on < 0 || on > 2) return ahr::fail(AHR_EINVAL, "on must be 0, 1 or 2");
    ahr::g_on = on;
    return AHR_OK;
}

ahr_status ahr_profile_read(ahr_profile* out, int32_t reset) {
    if (!out) return ahr::fail(AHR_EINVAL, "out is NULL");
    try {
        std::lock_guard<std::mutex> lk(ahr::g_mu);
        ahr::drain_locked();
        // one destination per stage, in Stage order
        double* ms[ahr::kStageCount] = {&out->build_ms, &out->hints_ms, &out->norm_ms, &out->expand_ms,
                                        &out->hop_ms,   &out->relax_ms, &out->hpwl_ms, &out->mlp_ms,
                                        &out->wa_ms};
        int64_t* cnt[ahr::kStageCount] = {&out->build_calls,  &out->hints_calls, &out->norm_calls,
                                          &out->expand_calls, &out->hop_launches, &out->relax_calls,
                                          &out->hpwl_calls,   &out->mlp_calls,   &out->wa_calls};
        static_assert(ahr::kStageCount == 9, "one profile field per stage");
        for (int k = 0; k < ahr::kStageCount; ++k) {
            *ms[k] = ahr::g_ms[k];
            *cnt[k] = ahr::g_count[k];
        }
        out->hop_bytes = ahr::g_bytes[ahr::kStageHop];
        out->wa_bytes = ahr::g_bytes[ahr::kStageWa];
        if (reset) {
            for (int k = 0; k < ahr::kStageCount; ++k) ahr::g_ms[k] = 0, ahr::g_count[k] = 0, ahr::g_bytes[k] = 0;
        }
        return AHR_OK;
    } catch (const ahr::Error& e) {
        return ahr::fail(e.code, e.msg);
    }
}

}  // extern "C"
