// Per-kernel HIP-event timing of the library's own launches.
//
// While enabled, every tracked launch is bracketed by two events recorded on
// the stream it runs on; chaff_profile_read() waits for them and aggregates
// the elapsed times per kernel name.  Events come from a reusable pool, so
// steady-state profiling creates no new HIP objects.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "prof.hpp"

namespace chaff {

namespace {
struct Rec {
    int name;
    hipEvent_t a, b;
    ProfWork w;
};
std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<std::string> g_names;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_pool_used = 0;

hipEvent_t take_event() {
    if (g_pool_used == g_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_pool.push_back(e);
    }
    return g_pool[g_pool_used++];
}
int name_id(const char* n) {
    for (size_t i = 0; i < g_names.size(); ++i)
        if (g_names[i] == n) return (int)i;
    g_names.emplace_back(n);
    return (int)g_names.size() - 1;
}
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t st, ProfWork w) : st_(st) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return;
    if (hipEventRecord(a, st) != hipSuccess) return;
    rec_ = (int)g_recs.size();
    g_recs.push_back(Rec{name_id(name), a, b, w});
}

ProfScope::~ProfScope() {
    if (rec_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (rec_ < (int)g_recs.size()) (void)hipEventRecord(g_recs[rec_].b, st_);
}

}  // namespace chaff

using namespace chaff;

extern "C" {

chaff_status chaff_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (on) {
        g_recs.clear();
        g_pool_used = 0;
    }
    g_on.store(on ? 1 : 0);
    return CHAFF_OK;
}

int32_t chaff_profile_read(chaff_kernel_time* out, int32_t max_out) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<chaff_kernel_time> agg(g_names.size());
    for (size_t i = 0; i < g_names.size(); ++i) {
        std::memset(&agg[i], 0, sizeof(chaff_kernel_time));
        std::strncpy(agg[i].name, g_names[i].c_str(), sizeof(agg[i].name) - 1);
        agg[i].min_ms = 1e300;
    }
    for (const Rec& r : g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        chaff_kernel_time& k = agg[r.name];
        k.launches += 1;
        k.total_ms += ms;
        k.min_ms = std::min(k.min_ms, (double)ms);
        k.max_ms = std::max(k.max_ms, (double)ms);
        k.bytes += r.w.bytes;
        k.flops += r.w.flops;
    }
    int32_t n = 0;
    for (auto& k : agg) {
        if (k.launches == 0) continue;
        if (n < max_out && out) out[n] = k;
        ++n;
    }
    return std::min(n, max_out);
}

}  // extern "C"
