// prof.cpp -- HIP-event timing of kernel launches (tsqr_prof_* in tsqr.h).
#include "prof.h"

#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tsqr.h"

namespace tsqr {
namespace {

struct Rec {
    const char *tag;
    hipEvent_t a, b;
};

// The state below is shared by every host thread that launches library
// kernels (the request server enqueues mixed-precision solves from worker
// threads): g_mu guards it; g_on is read without the lock on the fast path.
std::mutex g_mu;
std::atomic<bool> g_on{false};
int g_suspend = 0;    // > 0 while a stream is being captured into a graph
std::string g_only;   // when not empty, only this tag is timed
std::vector<Rec> g_recs;       // events recorded since the last query
std::vector<hipEvent_t> g_pool;
struct Agg {
    std::string tag;
    int64_t launches = 0;
    double ms = 0.0;
};
std::vector<Agg> g_agg;

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

void drain() {
    for (Rec &r : g_recs) {
        float ms = 0.f;
        if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            Agg *a = nullptr;
            for (Agg &x : g_agg)
                if (x.tag == r.tag) a = &x;
            if (!a) {
                g_agg.push_back(Agg{r.tag, 0, 0.0});
                a = &g_agg.back();
            }
            a->launches += 1;
            a->ms += ms;
        }
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_recs.clear();
}

}  // namespace

void prof_suspend(bool on) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_suspend += on ? 1 : -1;
}

int prof_begin(const char *tag, hipStream_t st) {
    if (!g_on.load(std::memory_order_relaxed)) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_suspend > 0) return -1;
    if (!g_only.empty() && g_only != tag) return -1;
    if (g_recs.size() > 20000) drain();
    Rec r{tag, get_event(), get_event()};
    if (r.a) hipEventRecord(r.a, st);
    g_recs.push_back(r);
    return (int)g_recs.size() - 1;
}

void prof_end(int slot, hipStream_t st) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if (slot >= (int)g_recs.size()) return;
    if (g_recs[slot].b) hipEventRecord(g_recs[slot].b, st);
}

}  // namespace tsqr

extern "C" {

TSQR_API int tsqr_prof_enable(int on) {
    std::lock_guard<std::mutex> lock(tsqr::g_mu);
    tsqr::drain();
    tsqr::g_agg.clear();
    tsqr::g_on = on != 0;
    return 0;
}

TSQR_API int tsqr_prof_only(const char *tag) {
    std::lock_guard<std::mutex> lock(tsqr::g_mu);
    tsqr::g_only = tag ? tag : "";
    return 0;
}

TSQR_API int tsqr_prof_query(int i, const char **name, int64_t *launches, double *ms) {
    std::lock_guard<std::mutex> lock(tsqr::g_mu);
    tsqr::drain();
    if (i < 0 || i >= (int)tsqr::g_agg.size()) return -1;
    if (name) *name = tsqr::g_agg[i].tag.c_str();
    if (launches) *launches = tsqr::g_agg[i].launches;
    if (ms) *ms = tsqr::g_agg[i].ms;
    return 0;
}

}  // extern "C"
