// server.cpp -- the least-squares request server (tsqr_server_* in tsqr.h).
//
// One host thread drives it.  Requests queue in arrival order; progress()
// retires the ones whose completion event has fired and admits queued ones
// while a slot is free and their device memory fits the arena:
//   new matrix:    [A ->] workspace, tsqr_factor, B ->, tsqr_lsq_solve, -> X
//   cached matrix: B ->, tsqr_lsq_solve, -> X      (same stream as the factor,
//                                                    which orders the users of
//                                                    its least-squares scratch)
// Each admitted request runs on one of several HIP streams, so copies and
// kernels of different requests overlap on the device.  Device memory comes
// from one arena (first-fit free list with coalescing); when a request does
// not fit, idle cached factors are evicted least recently used first, and
// younger requests that do fit may be admitted past it while it has waited
// less than the bypass window.
//
// A mixed-precision solve reads a convergence flag back after every
// refinement sweep, so it blocks the thread that enqueues it.  Its solve is
// therefore enqueued by a worker thread of its own (one per admitted mixed
// request); the driving thread keeps retiring and admitting meanwhile.  The
// solves of one cached factor share its workspace and are serialised by the
// entry's lock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tsqr.h"

namespace {

constexpr size_t kAl = 256;

size_t up(size_t x) { return (x + kAl - 1) / kAl * kAl; }

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
public:
    void init(size_t size) {
        size_ = size;
        free_.clear();
        free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Entry {
    int64_t matrix_id = 0, m = 0, n = 0;
    size_t off = 0, bytes = 0;      // workspace (+ A for mixed factors)
    size_t ws_off = 0, ws_bytes = 0;
    size_t a_off = 0;               // A (mixed: inside this entry)
    tsqr_factors f = nullptr;
    int stream = 0;
    int refs = 0;
    uint64_t last_use = 0;
    std::shared_ptr<std::mutex> solve_mu;   // serialises solves on this factor's workspace
};

// A mixed-precision solve enqueued by a worker thread.  state: 0 while the
// worker runs, 1 once the solve, the copies back and the completion event
// are enqueued, -1 when one of them failed (rc).
struct Job {
    std::thread th;
    std::atomic<int> state{0};
    int rc = 0;
};

struct Req {
    tsqr_request r{};
    int state = 0;                  // 0 queued, 1 running, 2 done, < 0 error
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t io_off = 0, io_bytes = 0;
    int64_t entry = -1;             // matrix id of its cache entry
    int stream = 0;
    hipEvent_t ev = nullptr;
    std::unique_ptr<Job> job;       // mixed precision: the worker enqueueing the solve
};

}  // namespace

struct tsqr_server_s {
    tsqr_server_opts o{};
    char *base = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    std::vector<hipEvent_t> ev_pool;
    std::deque<Req> reqs;           // a deque: references stay valid while requests are appended
    int device = 0;
    std::deque<int64_t> queue;
    std::vector<int64_t> running;
    std::unordered_map<int64_t, Entry> cache;
    std::unordered_map<int64_t, std::pair<int64_t, int64_t>> shapes;   // matrix id -> (m, n)
    uint64_t tick = 0;
    tsqr_server_stats st{};
    double t_last = 0;
};

namespace {

tsqr_opts factor_opts(const tsqr_server_s *S) {
    tsqr_opts o;
    tsqr_default_opts(&o);
    o.prec = S->o.prec;
    o.tree = S->o.tree;
    o.lsq_max_rhs = 8;
    o.route_kappa = S->o.route_kappa;
    return o;
}

void account(tsqr_server_s *S) {
    const double t = now_s();
    if (S->t_last > 0) {
        const double dt = t - S->t_last;
        if (!S->running.empty()) S->st.busy_seconds += dt;
        S->st.byte_seconds += dt * (double)S->arena.used();
    }
    S->t_last = t;
    S->st.bytes_in_use = S->arena.used();
    S->st.bytes_peak = std::max(S->st.bytes_peak, S->arena.used());
}

void drop_entry(tsqr_server_s *S, int64_t id) {
    auto it = S->cache.find(id);
    if (it == S->cache.end()) return;
    if (it->second.f) tsqr_free(it->second.f);
    S->arena.release(it->second.off, it->second.bytes);
    S->cache.erase(it);
}

// Drops the least recently used idle cached factor other than `keep` (the
// matrix the admitting request is about to use, whose entry must survive the
// admission); false when there is none.
bool evict_one(tsqr_server_s *S, int64_t keep) {
    int64_t victim = -1;
    uint64_t oldest = ~0ull;
    for (auto &kv : S->cache)
        if (kv.first != keep && kv.second.refs == 0 && kv.second.last_use < oldest) {
            oldest = kv.second.last_use;
            victim = kv.first;
        }
    if (victim < 0) return false;
    drop_entry(S, victim);
    S->st.evictions += 1;
    return true;
}

size_t io_bytes(const tsqr_server_s *S, const tsqr_request &r, bool with_a) {
    size_t b = up(sizeof(double) * r.m * r.k) + up(sizeof(double) * r.n * r.k) + up(sizeof(double) * 8) +
               up(sizeof(int32_t));
    if (with_a) b += up(sizeof(double) * r.m * r.n);
    (void)S;
    return b;
}

size_t entry_bytes(const tsqr_server_s *S, const tsqr_request &r, size_t *ws) {
    tsqr_opts o = factor_opts(S);
    *ws = tsqr_workspace_bytes(r.m, r.n, &o);
    size_t b = up(*ws);
    if (S->o.prec == TSQR_MIXED) b += up(sizeof(double) * r.m * r.n);
    return b;
}

void fail(tsqr_server_s *S, Req &q, int code) {
    q.state = code;
    q.t_done = now_s();
    S->st.failed += 1;
}

// The solve of an admitted request and the copies of its results back to
// the host, then its completion event, all on `st`.
int enqueue_solve(tsqr_factors f, const double *Adev, const tsqr_request &r, double *B, double *X,
                  double *res, int32_t *info, hipEvent_t ev, hipStream_t st) {
    int rc = tsqr_lsq_solve(f, Adev, r.m, r.k, B, r.m, X, r.n, res, info, st);
    if (!rc && (hipMemcpyAsync(r.X, X, sizeof(double) * r.n * r.k, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(r.resid, res, sizeof(double) * r.k, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(r.info, info, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess))
        rc = -1000;
    if (!rc && hipEventRecord(ev, st) != hipSuccess) rc = -1000;
    return rc;
}

// Tries to admit request q; returns 1 admitted, 0 must wait, -1 failed.
int admit(tsqr_server_s *S, int64_t ticket) {
    Req &q = S->reqs[ticket];
    const tsqr_request &r = q.r;
    const bool mixed = S->o.prec == TSQR_MIXED;
    auto hit = S->cache.find(r.matrix_id);
    bool have = hit != S->cache.end();
    size_t ws = 0, eb = 0, ib = 0;
    size_t io_off = 0, e_off = 0;
    for (;;) {
        const bool a_in_io = !have && !mixed;   // FP64 factors do not keep A
        eb = have ? 0 : entry_bytes(S, r, &ws);
        ib = io_bytes(S, r, a_in_io);
        if (!have && ws == 0) return -1;
        bool placed = false;
        for (;;) {
            bool ok_io = S->arena.alloc(ib, &io_off);
            bool ok_e = ok_io && (have || S->arena.alloc(eb, &e_off));
            if (ok_io && ok_e) {
                placed = true;
                break;
            }
            if (ok_io) S->arena.release(io_off, ib);
            if (!evict_one(S, r.matrix_id)) break;
        }
        if (placed) break;
        // the cached factor of this very matrix can be what is in the way
        // (it may split the free space): when it is idle, drop it and admit
        // the request as a new matrix
        if (have && hit->second.refs == 0) {
            drop_entry(S, r.matrix_id);
            S->st.evictions += 1;
            have = false;
            continue;
        }
        return S->running.empty() ? -1 : 0;
    }
    const bool a_in_io = !have && !mixed;
    hipStream_t st;
    int si;
    if (have) {
        si = hit->second.stream;
    } else {
        si = (int)(std::min_element(S->stream_load.begin(), S->stream_load.end()) - S->stream_load.begin());
    }
    st = S->streams[si];
    char *io = S->base + io_off;
    double *B = reinterpret_cast<double *>(io);
    double *X = reinterpret_cast<double *>(io + up(sizeof(double) * r.m * r.k));
    double *res = reinterpret_cast<double *>(reinterpret_cast<char *>(X) + up(sizeof(double) * r.n * r.k));
    int32_t *info = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(res) + up(sizeof(double) * 8));
    double *Aio = reinterpret_cast<double *>(reinterpret_cast<char *>(info) + up(sizeof(int32_t)));
    int rc = 0;
    const double *Adev = nullptr;
    if (!have) {
        Entry e;
        e.matrix_id = r.matrix_id;
        e.m = r.m;
        e.n = r.n;
        e.off = e_off;
        e.bytes = eb;
        e.ws_off = e_off;
        e.ws_bytes = ws;
        e.stream = si;
        e.solve_mu = std::make_shared<std::mutex>();
        double *Ad = a_in_io ? Aio : reinterpret_cast<double *>(S->base + e_off + up(ws));
        e.a_off = (size_t)(reinterpret_cast<char *>(Ad) - S->base);
        if (hipMemcpyAsync(Ad, r.A, sizeof(double) * r.m * r.n, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = -1000;
        tsqr_opts o = factor_opts(S);
        if (!rc) rc = tsqr_factor(r.m, r.n, Ad, r.m, &o, S->base + e.ws_off, ws, st, &e.f);
        if (rc) {
            hipStreamSynchronize(st);
            S->arena.release(io_off, ib);
            S->arena.release(e_off, eb);
            fail(S, q, rc);
            return -1;
        }
        Adev = Ad;
        S->cache.emplace(r.matrix_id, e);
        hit = S->cache.find(r.matrix_id);
    } else {
        S->st.cache_hits += 1;
        Adev = mixed ? reinterpret_cast<const double *>(S->base + hit->second.a_off) : nullptr;
    }
    Entry &E = hit->second;
    if (hipMemcpyAsync(B, r.B, sizeof(double) * r.m * r.k, hipMemcpyHostToDevice, st) != hipSuccess) rc = -1000;
    if (!rc) {
        if (!S->ev_pool.empty()) {
            q.ev = S->ev_pool.back();
            S->ev_pool.pop_back();
        } else if (hipEventCreateWithFlags(&q.ev, hipEventDisableTiming) != hipSuccess) {
            q.ev = nullptr;
            rc = -1000;
        }
    }
    if (!rc && mixed) {
        // the worker enqueues the blocking solve; this thread goes on
        auto job = std::make_unique<Job>();
        Job *jp = job.get();
        const tsqr_request rr = r;
        const tsqr_factors f = E.f;
        const std::shared_ptr<std::mutex> mu = E.solve_mu;
        const hipEvent_t ev = q.ev;
        const int dev = S->device;
        try {
            jp->th = std::thread([jp, rr, f, mu, Adev, B, X, res, info, ev, st, dev]() {
                int wrc = hipSetDevice(dev) == hipSuccess ? 0 : -1000;
                if (!wrc) {
                    std::lock_guard<std::mutex> lock(*mu);
                    wrc = enqueue_solve(f, Adev, rr, B, X, res, info, ev, st);
                }
                jp->rc = wrc;
                jp->state.store(wrc ? -1 : 1, std::memory_order_release);
            });
            q.job = std::move(job);
        } catch (...) {
            rc = -1000;
        }
    } else if (!rc) {
        rc = enqueue_solve(E.f, Adev, r, B, X, res, info, q.ev, st);
    }
    if (rc) {
        // the stream may still read the buffers: wait before releasing them
        hipStreamSynchronize(st);
        S->arena.release(io_off, ib);
        if (q.ev) S->ev_pool.push_back(q.ev);
        q.ev = nullptr;
        if (!have && E.refs == 0) drop_entry(S, r.matrix_id);
        fail(S, q, rc);
        return -1;
    }
    E.refs += 1;
    E.last_use = ++S->tick;
    q.state = 1;
    q.t_admit = now_s();
    q.io_off = io_off;
    q.io_bytes = ib;
    q.entry = r.matrix_id;
    q.stream = si;
    S->stream_load[si] += 1;
    S->running.push_back(ticket);
    return 1;
}

int retire(tsqr_server_s *S, bool block_one) {
    int done = 0;
    for (size_t i = 0; i < S->running.size();) {
        Req &q = S->reqs[S->running[i]];
        const bool block = block_one && done == 0 && i == 0;
        int job_rc = 0;
        if (q.job) {
            // a mixed solve: its event means something only once the worker
            // has enqueued everything
            if (block && q.job->state.load(std::memory_order_acquire) == 0) q.job->th.join();
            const int js = q.job->state.load(std::memory_order_acquire);
            if (js == 0) {
                ++i;
                continue;
            }
            if (q.job->th.joinable()) q.job->th.join();
            if (js < 0) {
                job_rc = q.job->rc ? q.job->rc : -1000;
                hipStreamSynchronize(S->streams[q.stream]);   // nothing may still read its buffers
            }
        }
        hipError_t e = hipSuccess;
        if (!job_rc) e = block ? hipEventSynchronize(q.ev) : hipEventQuery(q.ev);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        q.job.reset();
        q.t_done = now_s();
        q.state = job_rc ? job_rc : ((e == hipSuccess) ? 2 : -1000 - (int)e);
        if (q.state == 2) S->st.completed += 1;
        else S->st.failed += 1;
        S->ev_pool.push_back(q.ev);
        q.ev = nullptr;
        S->arena.release(q.io_off, q.io_bytes);
        S->stream_load[q.stream] -= 1;
        auto it = S->cache.find(q.entry);
        if (it != S->cache.end()) {
            it->second.refs -= 1;
            if (!S->o.cache && it->second.refs == 0) drop_entry(S, q.entry);
        }
        S->running.erase(S->running.begin() + i);
        ++done;
    }
    return done;
}

// Admits queued requests in arrival order while slots are free.  A request
// whose memory does not fit yet stays queued, and younger ones that fit are
// admitted past it until it has waited the bypass window; from then on
// nothing is admitted past it, so the memory that frees up goes to it.
void admit_queued(tsqr_server_s *S) {
    const double window = S->o.bypass_ms < 0 ? 0.0 : (S->o.bypass_ms == 0 ? 100.0 : S->o.bypass_ms) * 1e-3;
    for (auto it = S->queue.begin(); it != S->queue.end() && (int)S->running.size() < S->o.max_inflight;) {
        const int64_t t = *it;
        const int a = admit(S, t);
        if (a == 0) {
            if (now_s() - S->reqs[t].t_submit >= window) break;
            ++it;
            continue;
        }
        if (a < 0 && S->reqs[t].state == 0) fail(S, S->reqs[t], TSQR_ERR_WORKSPACE);
        it = S->queue.erase(it);
    }
}

}  // namespace

extern "C" {

TSQR_API double tsqr_server_now(void) { return now_s(); }

TSQR_API void tsqr_server_default_opts(tsqr_server_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->hbm_budget = (size_t)64 << 30;
    o->streams = 4;
    o->max_inflight = 16;
    o->cache = 1;
    o->prec = TSQR_F64;
    o->tree = TSQR_TREE_BINARY;
    o->route_kappa = 1e4;
}

TSQR_API int tsqr_server_create(const tsqr_server_opts *o, tsqr_server *out) {
    if (!out) return -2;
    *out = nullptr;
    tsqr_server_opts d;
    tsqr_server_default_opts(&d);
    if (!o) o = &d;
    if (o->hbm_budget < ((size_t)1 << 20) || o->streams < 1 || o->streams > 64 || o->max_inflight < 1 ||
        (o->prec != TSQR_F64 && o->prec != TSQR_MIXED) || !(o->route_kappa >= 0.0) ||
        (o->tree != TSQR_TREE_FLAT && o->tree != TSQR_TREE_BINARY && o->tree != TSQR_TREE_QUAD &&
         o->tree != TSQR_TREE_XCD))
        return -1;
    tsqr_server_s *S = new (std::nothrow) tsqr_server_s;
    if (!S) return TSQR_ERR_WORKSPACE;
    S->o = *o;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, o->hbm_budget);
    if (e != hipSuccess) {
        delete S;
        return -1000 - (int)e;
    }
    S->base = static_cast<char *>(p);
    S->arena.init(o->hbm_budget);
    if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
    for (int i = 0; i < o->streams; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : S->streams) hipStreamDestroy(x);
            hipFree(S->base);
            delete S;
            return -1000 - (int)e;
        }
        S->streams.push_back(st);
    }
    S->stream_load.assign(o->streams, 0);
    *out = S;
    return 0;
}

TSQR_API int64_t tsqr_server_submit(tsqr_server S, const tsqr_request *r) {
    if (!S || !r) return -1;
    if (r->n < 1 || r->n > 256 || r->m < r->n || r->m > 2147483647LL || r->k < 1 || r->k > 8) return -2;
    if (!r->A || !r->B || !r->X || !r->resid || !r->info) return -3;
    auto sh = S->shapes.find(r->matrix_id);
    if (sh != S->shapes.end() && (sh->second.first != r->m || sh->second.second != r->n)) return -4;
    size_t ws = 0;
    const size_t need = entry_bytes(S, *r, &ws) + io_bytes(S, *r, true);
    if (ws == 0) return -2;
    if (need > S->arena.size()) return TSQR_ERR_WORKSPACE;
    S->shapes[r->matrix_id] = {r->m, r->n};
    S->reqs.emplace_back();
    Req &q = S->reqs.back();
    q.r = *r;
    q.t_submit = now_s();
    const int64_t t = (int64_t)S->reqs.size() - 1;
    S->queue.push_back(t);
    S->st.submitted += 1;
    return t;
}

TSQR_API int tsqr_server_progress(tsqr_server S, int wait) {
    if (!S) return -1;
    account(S);
    int done = retire(S, false);
    admit_queued(S);
    if (wait && done == 0 && !S->running.empty()) {
        account(S);
        retire(S, true);
        admit_queued(S);
    }
    account(S);
    return (int)(S->queue.size() + S->running.size());
}

TSQR_API int tsqr_server_status(tsqr_server S, int64_t t) {
    if (!S || t < 0 || t >= (int64_t)S->reqs.size()) return -1;
    const int s = S->reqs[t].state;
    return s == 2 ? 1 : (s < 0 ? s : 0);
}

TSQR_API int tsqr_server_times(tsqr_server S, int64_t t, double *a, double *b, double *c) {
    if (!S || t < 0 || t >= (int64_t)S->reqs.size()) return -1;
    const Req &q = S->reqs[t];
    if (a) *a = q.t_submit;
    if (b) *b = q.t_admit;
    if (c) *c = q.t_done;
    return 0;
}

TSQR_API int tsqr_server_get_stats(tsqr_server S, tsqr_server_stats *st) {
    if (!S || !st) return -1;
    *st = S->st;
    return 0;
}

TSQR_API int tsqr_server_free(tsqr_server S) {
    if (!S) return 0;
    while (tsqr_server_progress(S, 1) > 0) {
    }
    for (auto &kv : S->cache)
        if (kv.second.f) tsqr_free(kv.second.f);
    S->cache.clear();
    for (hipEvent_t e : S->ev_pool) hipEventDestroy(e);
    for (hipStream_t st : S->streams) hipStreamDestroy(st);
    hipFree(S->base);
    delete S;
    return 0;
}

}  // extern "C"
