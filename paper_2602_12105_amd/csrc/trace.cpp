// Kernel timing with hipEvents (dgo_trace_*): a measurement aid, not part of
// the method. Events come from a recycled pool; records are resolved lazily.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace dgo {
namespace {

struct Rec {
    std::string name;
    hipEvent_t e0, e1;
};

struct Agg {
    int64_t count = 0;
    double total = 0, mn = 1e300, mx = 0;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::string g_filter;
std::vector<hipEvent_t> g_pool;
std::vector<Rec> g_pending;
std::map<std::string, Agg> g_agg;

void add_locked(const Rec &r, float ms) {
    Agg &a = g_agg[r.name];
    a.count += 1;
    a.total += ms;
    a.mn = std::min(a.mn, (double)ms);
    a.mx = std::max(a.mx, (double)ms);
}

// Resolve the oldest pending records whose stop event has already completed
// (non-blocking), so the events come back to the pool while the device is
// still working and no event is created inside a timed loop once the pool
// has reached the depth of work in flight.
void recycle_completed_locked() {
    size_t n = 0;
    while (n < g_pending.size()) {
        const hipError_t q = hipEventQuery(g_pending[n].e1);
        if (q != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        ++n;
    }
    for (size_t i = 0; i < n; ++i) {
        Rec &r = g_pending[i];
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess)
            add_locked(r, ms);
        else
            (void)hipGetLastError();
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_pending.erase(g_pending.begin(), g_pending.begin() + (std::ptrdiff_t)n);
}

hipEvent_t take_event() {
    if (g_pool.empty()) recycle_completed_locked();
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void resolve_locked() {
    for (Rec &r : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            add_locked(r, ms);
        } else {
            (void)hipGetLastError();
        }
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_pending.clear();
}

}  // namespace

TraceScope::TraceScope(const char *n, hipStream_t s) : name(n), stream(s) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_filter.empty() && !strstr(n, g_filter.c_str())) return;
    e0 = take_event();
    e1 = take_event();
    if (!e0 || !e1) {
        if (e0) g_pool.push_back(e0);
        if (e1) g_pool.push_back(e1);
        e0 = e1 = nullptr;
        return;
    }
    (void)hipEventRecord(e0, s);
}

TraceScope::~TraceScope() {
    if (!e0) return;
    (void)hipEventRecord(e1, stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({name, e0, e1});
    if (g_pending.size() > 4096) resolve_locked();
}

TracePair::TracePair(const char *n) : name(n) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_filter.empty() && !strstr(n, g_filter.c_str())) return;
    e0 = take_event();
    e1 = take_event();
    if (!e0 || !e1) {
        if (e0) g_pool.push_back(e0);
        if (e1) g_pool.push_back(e1);
        e0 = e1 = nullptr;
    }
}

TracePair::~TracePair() {
    if (!e0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({name, e0, e1});
    if (g_pending.size() > 4096) resolve_locked();
}

bool trace_active() { return g_on.load(std::memory_order_relaxed); }

}  // namespace dgo

using namespace dgo;

extern "C" dgo_status dgo_trace_enable(int32_t on, const char *filter) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_filter = filter ? filter : "";
    g_on.store(on != 0);
    return DGO_OK;
}

extern "C" dgo_status dgo_trace_read(dgo_trace_entry *out, int32_t cap, int32_t *n) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_locked();
    std::vector<std::pair<std::string, Agg>> v(g_agg.begin(), g_agg.end());
    std::sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.second.total > b.second.total; });
    if (n) *n = (int32_t)v.size();
    for (int32_t i = 0; out && i < cap && i < (int32_t)v.size(); ++i) {
        memset(&out[i], 0, sizeof(out[i]));
        strncpy(out[i].name, v[i].first.c_str(), sizeof(out[i].name) - 1);
        out[i].count = v[i].second.count;
        out[i].total_ms = v[i].second.total;
        out[i].min_ms = v[i].second.mn;
        out[i].max_ms = v[i].second.mx;
    }
    return DGO_OK;
}

extern "C" void dgo_trace_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_locked();
    g_agg.clear();
}
