// batch.cpp -- batched TSQR + least squares (tsqr_batch_* and tsqr_autotune
// in tsqr.h).
//
// Each matrix gets its own single-panel plan (domains, chunks, tree levels)
// from the tuning table; the batch is then a fixed sequence of launches, each
// covering every matrix that has work at that step:
//   leaf QR per slot width class (ns = 1, 2, 4), tree levels per class,
//   sign normalisation, F = b, sweep 0 (Q^T F, solve), and for the mixed
//   matrices `refine_sweeps` refinement sweeps whose kernels skip matrices
//   that have converged, then the outputs.
// The descriptors and index lists live at the front of the caller's
// workspace, so the sequence can be captured once into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "prof.h"

namespace {

using tsqr::BMat;
using tsqr::Plan;

constexpr int64_t kTuneMb[] = {512, 1024, 2048, 4096, 8192};
constexpr int kTuneTree[] = {TSQR_TREE_BINARY, TSQR_TREE_QUAD, TSQR_TREE_FLAT};
constexpr int kNClass[] = {8, 16, 32, 64};

thread_local int g_bad_item = -1;

size_t align_up(size_t x) { return (x + tsqr::kAlign - 1) / tsqr::kAlign * tsqr::kAlign; }

int n_class(int64_t n) {
    for (int c : kNClass)
        if (n <= c) return c;
    return 64;
}

// (row_block, tree) of a matrix from the table: the entry of its precision
// with the smallest n_max >= n; the batch default otherwise.
void lookup(const tsqr_tune_entry *tune, int ntune, int64_t n, int prec, int64_t *mb, int *tree) {
    *mb = TSQR_BATCH_DEFAULT_ROW_BLOCK;
    *tree = TSQR_TREE_BINARY;
    int best = 1 << 30;
    for (int i = 0; i < ntune; ++i) {
        const tsqr_tune_entry &e = tune[i];
        if (e.prec != prec || e.n_max < n || e.n_max >= best) continue;
        best = e.n_max;
        *mb = e.row_block;
        *tree = e.tree;
    }
    if (*mb < n) *mb = n;
}

bool item_ok(const tsqr_batch_item &it) {
    return it.n >= 1 && it.n <= tsqr::kMaxPanel && it.m >= it.n && it.m <= 2147483647LL &&
           (it.prec == TSQR_F64 || it.prec == TSQR_MIXED);
}

struct MatPlan {
    Plan plan;
    size_t off = 0, bytes = 0;   // region of this matrix in the workspace
};

int plan_matrix(const tsqr_batch_item &it, int64_t mb, int tree, MatPlan *mp) {
    tsqr_opts o;
    tsqr_default_opts(&o);
    o.row_block = mb;
    o.tree = tree;
    o.prec = it.prec;
    o.lsq_max_rhs = 1;
    int rc = tsqr::make_plan(it.m, it.n, &o, &mp->plan);
    if (rc) return rc;
    const tsqr::Panel &p = mp->plan.panels[0];
    const size_t m = (size_t)it.m, n = (size_t)it.n, nn = n * n * sizeof(double);
    const size_t nb = (size_t)tsqr::resid_blocks(it.m);
    size_t b = 0;
    b += align_up((it.prec ? sizeof(float) : sizeof(double)) * m * n);       // V
    b += align_up(nn * (size_t)p.total_chunks);                              // Tc
    b += 2 * align_up(nn * (size_t)p.P);                                     // Rdom, Tnode
    b += align_up(sizeof(double) * n);                                       // dsign
    b += align_up(sizeof(double) * m);                                       // F
    if (it.prec) b += align_up(sizeof(double) * m);                          // Rr
    b += align_up(sizeof(double) * n);                                       // Xw
    if (it.prec) b += align_up(sizeof(double) * nb * n);                     // gpart
    b += align_up(sizeof(double) * 2 * nb);                                  // rpart
    b += align_up(sizeof(double) * 3 + sizeof(int32_t) * 2);                 // hist, status
    b += 2 * align_up(sizeof(double) * n * (size_t)p.total_chunks);         // Pc, Zc
    mp->bytes = b;
    return 0;
}

size_t header_bytes(int count) {
    return align_up(sizeof(BMat) * (size_t)count) + align_up(sizeof(int) * (size_t)count * 5);
}

// Group of matrices launched together, with the grid extents it needs.
struct Group {
    int list_off = 0;            // offset (in ints) of its index list
    int cnt = 0;
    int ns = 0;
    int64_t maxP = 0, maxNb = 0, maxM = 0, maxChunks = 0;
    int maxLev = 0;
    std::vector<int64_t> up;     // per bottom-up step: largest chain count
    std::vector<int64_t> down;   // per top-down step
};

}  // namespace

struct tsqr_batch_s {
    int count = 0;
    std::vector<BMat> host;          // descriptors (kept alive for the async upload)
    std::vector<int> lists;
    std::vector<Group> cls;          // slot-width classes (leaf and tree factor)
    Group all, mixed;
    std::vector<int64_t> mb;
    std::vector<int> tree;
    std::vector<int64_t> P;
    BMat *dmats = nullptr;
    int *dlists = nullptr;
    int sweeps = 0;
    double tol = 1e-14;
    int launches = 0;
    hipGraphExec_t exec = nullptr;
};

namespace {

void fill_group(Group &g, const std::vector<int> &idx, const tsqr_batch_s &B, int off) {
    g.list_off = off;
    g.cnt = (int)idx.size();
    for (int j : idx) {
        const BMat &M = B.host[j];
        g.maxP = std::max(g.maxP, M.pa.P);
        g.maxNb = std::max<int64_t>(g.maxNb, M.nb);
        g.maxM = std::max(g.maxM, M.pa.m);
        g.maxChunks = std::max(g.maxChunks, M.tchunks);
        g.maxLev = std::max(g.maxLev, M.nlev);
    }
    g.up.assign(g.maxLev, 0);
    g.down.assign(g.maxLev, 0);
    for (int j : idx) {
        const BMat &M = B.host[j];
        for (int L = 0; L < M.nlev; ++L) {
            g.up[L] = std::max(g.up[L], M.lev[L].chains);
            g.down[L] = std::max(g.down[L], M.lev[M.nlev - 1 - L].chains);
        }
    }
}

#define TRYB(call)                                       \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return -1000 - (int)e_;    \
    } while (0)

int enqueue(tsqr_batch_s *B, hipStream_t st, int *launches) {
    int nl = 0;
    const BMat *D = B->dmats;
    auto L = [&](const Group &g) { return B->dlists + g.list_off; };
    for (const Group &g : B->cls) {
        TRYB(tsqr::launch_leaf_b(D, L(g), g.cnt, g.maxP, g.ns, st));
        ++nl;
    }
    for (const Group &g : B->cls) {
        for (int lv = 0; lv < g.maxLev; ++lv) {
            TRYB(tsqr::launch_tree_b(D, L(g), g.cnt, g.up[lv], g.ns, lv, st));
            ++nl;
        }
        TRYB(tsqr::launch_tree_t_b(D, L(g), g.cnt, g.maxP, st));
        ++nl;
    }
    const Group &A = B->all;
    TRYB(tsqr::launch_sign_b(D, L(A), A.cnt, st));
    TRYB(tsqr::launch_lsq_init_b(D, L(A), A.cnt, (A.maxM + 2047) / 2048, st));
    TRYB(tsqr::launch_apply3_b(D, L(A), A.cnt, A.maxChunks, A.maxP, 1, 0, st));
    nl += 5;
    for (int s = 0; s < A.maxLev; ++s) {
        TRYB(tsqr::launch_tree_apply_b(D, L(A), A.cnt, A.up[s], 1, s, 0, st));
        ++nl;
    }
    TRYB(tsqr::launch_scale_b(D, L(A), A.cnt, 0, st));
    TRYB(tsqr::launch_refine_b(D, L(A), A.cnt, 0, B->tol, st));
    nl += 2;
    const Group &X = B->mixed;
    if (X.cnt > 0)
        for (int sw = 1; sw <= B->sweeps; ++sw) {
            // r += Q [h; d2]
            TRYB(tsqr::launch_scale_b(D, L(X), X.cnt, sw, st));
            for (int s = 0; s < X.maxLev; ++s)
                TRYB(tsqr::launch_tree_apply_b(D, L(X), X.cnt, X.down[s], 0, s, sw, st));
            TRYB(tsqr::launch_apply3_b(D, L(X), X.cnt, X.maxChunks, X.maxP, 0, sw, st));
            TRYB(tsqr::launch_axpy_b(D, L(X), X.cnt, (X.maxM + 2047) / 2048, sw, st));
            // f = b - r - A x, g = -A^T r (FP64), then Q^T f and the solve
            TRYB(tsqr::launch_resid_b(D, L(X), X.cnt, X.maxNb, sw, st));
            TRYB(tsqr::launch_apply3_b(D, L(X), X.cnt, X.maxChunks, X.maxP, 1, sw, st));
            for (int s = 0; s < X.maxLev; ++s)
                TRYB(tsqr::launch_tree_apply_b(D, L(X), X.cnt, X.up[s], 1, s, sw, st));
            TRYB(tsqr::launch_scale_b(D, L(X), X.cnt, sw, st));
            TRYB(tsqr::launch_refine_b(D, L(X), X.cnt, sw, B->tol, st));
            nl += 12 + 2 * X.maxLev;
        }
    TRYB(tsqr::launch_final_b(D, L(A), A.cnt, st));
    ++nl;
    if (launches) *launches = nl;
    return 0;
}

size_t workspace_for(int count, const tsqr_batch_item *items, const tsqr_tune_entry *tune, int ntune) {
    size_t total = header_bytes(count);
    for (int i = 0; i < count; ++i) {
        if (!item_ok(items[i])) {
            g_bad_item = i;
            return 0;
        }
        size_t best = 0;
        if (tune) {
            int64_t mb;
            int tr;
            lookup(tune, ntune, items[i].n, items[i].prec, &mb, &tr);
            MatPlan mp;
            if (plan_matrix(items[i], mb, tr, &mp)) {
                g_bad_item = i;
                return 0;
            }
            best = mp.bytes;
        } else {
            for (int64_t mb : kTuneMb)
                for (int tr : kTuneTree) {
                    MatPlan mp;
                    if (plan_matrix(items[i], std::max<int64_t>(mb, items[i].n), tr, &mp)) {
                        g_bad_item = i;
                        return 0;
                    }
                    best = std::max(best, mp.bytes);
                }
            MatPlan mp;   // the default plan too
            if (plan_matrix(items[i], std::max<int64_t>(TSQR_BATCH_DEFAULT_ROW_BLOCK, items[i].n),
                            TSQR_TREE_BINARY, &mp) == 0)
                best = std::max(best, mp.bytes);
        }
        total += best;
    }
    return total;
}

}  // namespace

extern "C" {

TSQR_API int tsqr_batch_bad_item(void) { return g_bad_item; }

TSQR_API size_t tsqr_batch_workspace_bytes(int count, const tsqr_batch_item *items,
                                           const tsqr_tune_entry *tune, int ntune) {
    g_bad_item = -1;
    if (count < 1 || !items || (tune && ntune < 0)) return 0;
    return workspace_for(count, items, tune, ntune);
}

TSQR_API int tsqr_batch_create(int count, const tsqr_batch_item *items, const tsqr_tune_entry *tune,
                               int ntune, int refine_sweeps, double refine_tol, void *dwork,
                               size_t work_bytes, void *stream, tsqr_batch *out) {
    g_bad_item = -1;
    if (!out) return -10;
    *out = nullptr;
    if (count < 1 || count > 65535) return -1;
    if (!items) return -2;
    if (tune && ntune < 0) return -3;
    if (refine_sweeps < 0 || !(refine_tol >= 0.0)) return -5;
    for (int i = 0; i < count; ++i) {
        const tsqr_batch_item &it = items[i];
        if (!item_ok(it) || !it.A || it.lda < it.m || !it.b || !it.R || !it.x || !it.resid || !it.info) {
            g_bad_item = i;
            return -2;
        }
    }
    if (!dwork || (reinterpret_cast<uintptr_t>(dwork) % tsqr::kAlign)) return TSQR_ERR_WORKSPACE;
    tsqr_batch_s *B = new (std::nothrow) tsqr_batch_s;
    if (!B) return TSQR_ERR_WORKSPACE;
    B->count = count;
    B->sweeps = refine_sweeps;
    B->tol = refine_tol;
    B->host.resize(count);
    B->mb.resize(count);
    B->tree.resize(count);
    B->P.resize(count);
    char *base = static_cast<char *>(dwork);
    size_t off = header_bytes(count);
    std::vector<int> by_ns[3], all_idx, mixed_idx;
    for (int i = 0; i < count; ++i) {
        const tsqr_batch_item &it = items[i];
        int64_t mb;
        int tr;
        lookup(tune, tune ? ntune : 0, it.n, it.prec, &mb, &tr);
        MatPlan mp;
        if (plan_matrix(it, mb, tr, &mp)) {
            g_bad_item = i;
            delete B;
            return -2;
        }
        if (off + mp.bytes > work_bytes) {
            delete B;
            return TSQR_ERR_WORKSPACE;
        }
        const tsqr::Panel &p = mp.plan.panels[0];
        BMat &M = B->host[i];
        std::memset(&M, 0, sizeof(M));
        M.A = it.A;
        M.lda = it.lda;
        M.b = it.b;
        M.R = it.R;
        M.x = it.x;
        M.resid = it.resid;
        M.info = it.info;
        const size_t m = (size_t)it.m, n = (size_t)it.n, nn = n * n * sizeof(double);
        const int nb = tsqr::resid_blocks(it.m);
        char *q = base + off;
        auto take = [&](size_t bytes) {
            char *at = q;
            q += align_up(bytes);
            return at;
        };
        if (it.prec) M.V32 = reinterpret_cast<float *>(take(sizeof(float) * m * n));
        else M.V = reinterpret_cast<double *>(take(sizeof(double) * m * n));
        M.Tc = reinterpret_cast<double *>(take(nn * (size_t)p.total_chunks));
        M.Rdom = reinterpret_cast<double *>(take(nn * (size_t)p.P));
        M.Tnode = reinterpret_cast<double *>(take(nn * (size_t)p.P));
        M.dsign = reinterpret_cast<double *>(take(sizeof(double) * n));
        M.F = reinterpret_cast<double *>(take(sizeof(double) * m));
        if (it.prec) M.Rr = reinterpret_cast<double *>(take(sizeof(double) * m));
        M.Xw = reinterpret_cast<double *>(take(sizeof(double) * n));
        if (it.prec) M.gpart = reinterpret_cast<double *>(take(sizeof(double) * (size_t)nb * n));
        M.rpart = reinterpret_cast<double *>(take(sizeof(double) * 2 * (size_t)nb));
        char *hs = take(sizeof(double) * 3 + sizeof(int32_t) * 2);
        M.hist = reinterpret_cast<double *>(hs);
        M.status = reinterpret_cast<int32_t *>(hs + 3 * sizeof(double));
        M.Pc = reinterpret_cast<double *>(take(sizeof(double) * n * (size_t)p.total_chunks));
        M.Zc = reinterpret_cast<double *>(take(sizeof(double) * n * (size_t)p.total_chunks));
        M.tchunks = p.total_chunks;
        off += mp.bytes;
        M.pa.m = p.m;
        M.pa.mb = p.mb;
        M.pa.P = p.P;
        M.pa.cpd = p.cpd;
        M.pa.chunk = p.chunk;
        M.pa.extra = p.extra;
        M.pa.wtab = nullptr;
        M.pa.maxch = p.maxch;
        M.pa.n = p.n;
        M.pa.ns = p.ns;
        M.prec = it.prec;
        M.nb = nb;
        auto lv = tsqr::tree_levels(p.P, p.tree);
        if ((int)lv.size() > tsqr::kMaxLevels) {
            g_bad_item = i;
            delete B;
            return -2;
        }
        M.nlev = (int)lv.size();
        for (int l = 0; l < M.nlev; ++l) M.lev[l] = tsqr::TreeArgs{lv[l].stride, lv[l].span, lv[l].chains, lv[l].width};
        B->mb[i] = p.mb;
        B->tree[i] = p.tree;
        B->P[i] = p.P;
        by_ns[p.ns == 1 ? 0 : (p.ns == 2 ? 1 : 2)].push_back(i);
        all_idx.push_back(i);
        if (it.prec) mixed_idx.push_back(i);
    }
    // index lists: classes, all, mixed
    int loff = 0;
    for (int c = 0; c < 3; ++c) {
        if (by_ns[c].empty()) continue;
        Group g;
        fill_group(g, by_ns[c], *B, loff);
        g.ns = 1 << c;
        B->cls.push_back(g);
        B->lists.insert(B->lists.end(), by_ns[c].begin(), by_ns[c].end());
        loff += (int)by_ns[c].size();
    }
    fill_group(B->all, all_idx, *B, loff);
    B->lists.insert(B->lists.end(), all_idx.begin(), all_idx.end());
    loff += (int)all_idx.size();
    fill_group(B->mixed, mixed_idx, *B, loff);
    B->lists.insert(B->lists.end(), mixed_idx.begin(), mixed_idx.end());
    B->dmats = reinterpret_cast<BMat *>(base);
    B->dlists = reinterpret_cast<int *>(base + align_up(sizeof(BMat) * (size_t)count));
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(B->dmats, B->host.data(), sizeof(BMat) * (size_t)count,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->dlists, B->lists.data(), sizeof(int) * B->lists.size(), hipMemcpyHostToDevice,
                           st);
    // the host copies must outlive the asynchronous upload
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete B;
        return -1000 - (int)e;
    }
    *out = B;
    return 0;
}

TSQR_API int tsqr_batch_run(tsqr_batch B, int use_graph, void *stream) {
    if (!B) return -1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!use_graph) return enqueue(B, st, &B->launches);
    if (!st) return -3;
    if (!B->exec) {
        hipGraph_t g = nullptr;
        TRYB(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        tsqr::prof_suspend(true);
        int rc = enqueue(B, st, &B->launches);
        tsqr::prof_suspend(false);
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return -1000 - (int)e;
        e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) {
            B->exec = nullptr;
            return -1000 - (int)e;
        }
    }
    TRYB(hipGraphLaunch(B->exec, st));
    return 0;
}

TSQR_API int tsqr_batch_plan(tsqr_batch B, int i, int64_t *row_block, int32_t *tree, int64_t *domains) {
    if (!B) return -1;
    if (i < 0 || i >= B->count) return -2;
    if (row_block) *row_block = B->mb[i];
    if (tree) *tree = B->tree[i];
    if (domains) *domains = B->P[i];
    return 0;
}

TSQR_API int tsqr_batch_launches(tsqr_batch B) {
    if (!B) return -1;
    if (B->launches == 0) {
        // count without launching: the sequence is fixed by the plan
        int nl = (int)B->cls.size();
        for (const Group &g : B->cls) nl += g.maxLev;
        nl += 7 + B->all.maxLev + 1;
        if (B->mixed.cnt > 0) nl += B->sweeps * (12 + 2 * B->mixed.maxLev);
        return nl;
    }
    return B->launches;
}

TSQR_API int tsqr_batch_free(tsqr_batch B) {
    if (!B) return 0;
    if (B->exec) hipGraphExecDestroy(B->exec);
    delete B;
    return 0;
}

TSQR_API int tsqr_autotune(int count, const tsqr_batch_item *items, int reps, void *dwork, size_t work_bytes,
                           void *stream, tsqr_tune_entry *out, int cap) {
    if (count < 1 || !items) return -1;
    if (reps < 1) return -3;
    if (!out) return -7;
    const size_t need = tsqr_batch_workspace_bytes(count, items, nullptr, 0);
    if (need == 0) return -2;
    if (!dwork || work_bytes < need) return TSQR_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the classes present in the batch
    std::vector<tsqr_tune_entry> table;
    for (int i = 0; i < count; ++i) {
        const int nc = n_class(items[i].n);
        bool seen = false;
        for (auto &e : table) seen |= (e.n_max == nc && e.prec == items[i].prec);
        if (!seen) table.push_back(tsqr_tune_entry{nc, items[i].prec, TSQR_BATCH_DEFAULT_ROW_BLOCK,
                                                   TSQR_TREE_BINARY, 0});
    }
    std::sort(table.begin(), table.end(), [](const tsqr_tune_entry &a, const tsqr_tune_entry &b) {
        return a.prec != b.prec ? a.prec < b.prec : a.n_max < b.n_max;
    });
    if ((int)table.size() > cap) return -8;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TRYB(hipEventCreate(&e0));
    TRYB(hipEventCreate(&e1));
    auto time_table = [&](const std::vector<tsqr_tune_entry> &t, float *ms) -> int {
        tsqr_batch b = nullptr;
        int rc = tsqr_batch_create(count, items, t.data(), (int)t.size(), 2, 1e-14, dwork, work_bytes,
                                   stream, &b);
        if (rc) return rc;
        rc = tsqr_batch_run(b, 0, stream);   // warm-up
        if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = -1000;
        for (int r = 0; r < reps && !rc; ++r) rc = tsqr_batch_run(b, 0, stream);
        if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = -1000;
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = -1000;
        if (!rc && hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = -1000;
        tsqr_batch_free(b);
        return rc;
    };
    int rc = 0;
    float best = 0.f;
    // stage 1: one setting for every class
    std::vector<tsqr_tune_entry> cur = table;
    bool first = true;
    for (int64_t mb : kTuneMb)
        for (int tr : kTuneTree) {
            std::vector<tsqr_tune_entry> t = table;
            for (auto &e : t) {
                e.row_block = mb;
                e.tree = tr;
            }
            float ms = 0.f;
            if ((rc = time_table(t, &ms))) goto done;
            if (first || ms < best) {
                best = ms;
                cur = t;
                first = false;
            }
        }
    // stage 2: each class's row block on its own, then its tree
    for (size_t c = 0; c < cur.size(); ++c) {
        for (int64_t mb : kTuneMb) {
            if (cur[c].row_block == mb) continue;
            std::vector<tsqr_tune_entry> t = cur;
            t[c].row_block = mb;
            float ms = 0.f;
            if ((rc = time_table(t, &ms))) goto done;
            if (ms < 0.99f * best) {
                best = ms;
                cur = t;
            }
        }
        for (int tr : kTuneTree) {
            if (cur[c].tree == tr) continue;
            std::vector<tsqr_tune_entry> t = cur;
            t[c].tree = tr;
            float ms = 0.f;
            if ((rc = time_table(t, &ms))) goto done;
            if (ms < 0.99f * best) {
                best = ms;
                cur = t;
            }
        }
    }
    for (size_t c = 0; c < cur.size(); ++c) out[c] = cur[c];
    rc = (int)cur.size();
done:
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
