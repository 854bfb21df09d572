// Per-launch kernel timing (ttsvd_profile_* in the C ABI).
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "profile.h"

namespace ttsvd {
namespace {

struct Rec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;  // none for records added with a duration
    double bytes = 0, flops = 0;
    double ms = -1.0;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local int g_open = -1;

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

}  // namespace

bool prof_on() { return g_on.load(std::memory_order_relaxed) != 0; }

void prof_add(const char *name, double ms, double bytes, double flops) {
    if (!prof_on()) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Rec r;
    r.name = name;
    r.ms = ms;
    r.bytes = bytes;
    r.flops = flops;
    g_recs.push_back(r);
}

void prof_begin(hipStream_t s, const char *name, double bytes, double flops) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Rec r;
    r.name = name;
    r.bytes = bytes;
    r.flops = flops;
    r.a = take_event();
    r.b = take_event();
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, s);
    g_recs.push_back(r);
    g_open = (int)g_recs.size() - 1;
}

void prof_end(hipStream_t s) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_open < 0 || g_open >= (int)g_recs.size()) return;
    (void)hipEventRecord(g_recs[g_open].b, s);
    g_open = -1;
}

}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

int ttsvd_profile_enable(int on) {
    g_on.store(on ? 1 : 0);
    return TTSVD_OK;
}

void ttsvd_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (Rec &r : g_recs) {
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_open = -1;
}

int ttsvd_profile_read(ttsvd_kernel_stat *stats, int max_stats, int *n_stats) {
    clear_error();
    if (!n_stats || (max_stats > 0 && !stats)) return set_error(TTSVD_EINVAL, "profile_read: NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::string, ttsvd_kernel_stat> agg;
    std::vector<std::string> order;
    for (const Rec &r : g_recs) {
        float ms = (float)r.ms;
        if (r.ms < 0) {
            hipError_t e = hipEventSynchronize(r.b);
            if (e != hipSuccess)
                return set_error(TTSVD_EHIP, "profile_read: %s", hipGetErrorString(e));
            e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess)
                return set_error(TTSVD_EHIP, "profile_read: %s", hipGetErrorString(e));
        }
        auto it = agg.find(r.name);
        if (it == agg.end()) {
            ttsvd_kernel_stat st;
            memset(&st, 0, sizeof(st));
            strncpy(st.name, r.name.c_str(), sizeof(st.name) - 1);
            it = agg.emplace(r.name, st).first;
            order.push_back(r.name);
        }
        it->second.launches += 1;
        it->second.total_ms += ms;
        it->second.bytes += r.bytes;
        it->second.flops += r.flops;
    }
    int n = 0;
    for (const std::string &k : order) {
        if (n < max_stats) stats[n] = agg[k];
        ++n;
    }
    *n_stats = n;
    return TTSVD_OK;
}

}  // extern "C"
