// pic_profile.hip -- optional per-kernel timing with HIP events.
//
// When enabled, every kernel the library launches is bracketed by two events
// recorded on the stream it is launched on; pic_profile_read() waits for the
// recorded events and returns per-kernel launch counts and total times.
// Single-threaded use: the library is driven from one host thread.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "pic_host.h"

namespace pic {

namespace {
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
bool g_on = false;
thread_local int g_suspended = 0;  // > 0 inside a call that must not create timing events
std::string g_only;  // when set, only launches of this kernel name are timed
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

ProfSuspend::ProfSuspend() { ++g_suspended; }
ProfSuspend::~ProfSuspend() { --g_suspended; }

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s), a_(nullptr) {
    if (!g_on || g_suspended) return;
    if (!g_only.empty() && g_only != name) return;
    a_ = get_event();
    if (a_) hipEventRecord((hipEvent_t)a_, s);
}

ProfScope::~ProfScope() {
    if (!g_on || !a_) return;
    hipEvent_t b = get_event();
    if (!b) return;
    hipEventRecord(b, s_);
    g_recs.push_back(Rec{name_, (hipEvent_t)a_, b});
}

}  // namespace pic

extern "C" {

pic_status pic_profile_enable(int32_t on) {
    pic::g_on = on != 0;
    return PIC_OK;
}

pic_status pic_profile_only(const char *name) {
    pic::g_only = name ? name : "";
    return PIC_OK;
}

int32_t pic_profile_read(pic_kernel_time *out, int32_t max_entries) {
    using namespace pic;
    std::vector<pic_kernel_time> agg;
    for (const Rec &r : g_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess) hipEventElapsedTime(&ms, r.a, r.b);
        pic_kernel_time *slot = nullptr;
        for (auto &k : agg)
            if (std::strncmp(k.name, r.name, sizeof(k.name)) == 0) slot = &k;
        if (!slot) {
            agg.push_back(pic_kernel_time{});
            slot = &agg.back();
            std::strncpy(slot->name, r.name, sizeof(slot->name) - 1);
        }
        slot->launches += 1;
        slot->total_ms += ms;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    const int32_t n = (int32_t)agg.size();
    if (out)
        for (int32_t i = 0; i < n && i < max_entries; ++i) out[i] = agg[i];
    return n;
}

}  // extern "C"
