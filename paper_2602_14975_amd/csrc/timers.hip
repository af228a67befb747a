// Optional HIP-event timing of named launch sites (diagnostics entry points
// of nnp.h).  When a site is enabled, each launch is bracketed by two events
// recorded on the launch's own stream; reading synchronises on the events and
// returns the summed device durations.
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.h"
#include "kernels.h"

namespace nnp {

namespace {
struct Site {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
std::mutex g_mu;
std::unordered_map<std::string, Site> g_sites;
bool g_any = false;
}  // namespace

ScopedTimer::ScopedTimer(const char* site, hipStream_t s, bool launch_events)
    : name(site), stream(s), by_launch(launch_events) {
    if (!g_any) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_sites.find(name);
    if (it == g_sites.end() || !it->second.on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    if (!by_launch && hipEventRecord(a, stream) != hipSuccess) return;
    active = true;
}

ScopedTimer::~ScopedTimer() {
    if (!active) return;
    if (!by_launch) (void)hipEventRecord(b, stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_sites[name].ev.emplace_back(a, b);
}

bool timers_active() { return g_any; }

}  // namespace nnp

using namespace nnp;

extern "C" nnp_status nnp_timer_enable(const char* site, int32_t on) {
    if (!site) {
        set_error("null site name");
        return NNP_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_sites[site].on = on != 0;
    g_any = false;
    for (auto& kv : g_sites) g_any |= kv.second.on;
    return NNP_OK;
}

extern "C" nnp_status nnp_timer_read(const char* site, double* total_ms, int64_t* launches, int32_t reset) {
    if (!site || !total_ms || !launches) {
        set_error("null argument");
        return NNP_EINVAL;
    }
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_sites.find(site);
        if (it != g_sites.end()) {
            ev = it->second.ev;
            if (reset) it->second.ev.clear();
        }
    }
    double tot = 0.0;
    for (auto& p : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess) {
            set_error("event timing failed");
            return NNP_EDEVICE;
        }
        tot += ms;
        if (reset) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
    *total_ms = tot;
    *launches = int64_t(ev.size());
    return NNP_OK;
}
