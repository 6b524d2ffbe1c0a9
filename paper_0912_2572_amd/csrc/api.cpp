// api.cpp -- the C ABI declared in include/tsqr.h.
//
// Every entry point validates its arguments on the host, then enqueues the
// kernels of kernels.h on the caller's stream.  No device memory is
// allocated here: the workspace, inputs and outputs belong to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "handle.h"
#include "kernels.h"
#include "plan.h"

namespace {

using tsqr::Panel;
using tsqr::PanelArgs;
using tsqr::Plan;
using tsqr::TreeArgs;

inline int hip_code(hipError_t e) { return -1000 - (int)e; }

PanelArgs panel_args(const Panel &p) {
    PanelArgs a;
    a.m = p.m;
    a.mb = p.mb;
    a.P = p.P;
    a.cpd = p.cpd;
    a.chunk = p.chunk;
    a.extra = p.extra;
    a.wtab = nullptr;
    a.maxch = p.maxch;
    a.n = p.n;
    a.ns = p.ns;
    return a;
}

// PanelArgs of a panel of the factor in workspace ws: a weighted partition's
// table is the workspace copy.
PanelArgs panel_args(const Panel &p, const char *ws) {
    PanelArgs a = panel_args(p);
    if (!p.wchunk0.empty()) a.wtab = reinterpret_cast<const int64_t *>(ws + p.off_wtab);
    return a;
}

template <typename T>
T *at(const tsqr_factors_s *f, size_t off) {
    return reinterpret_cast<T *>(f->ws + off);
}

#define TRY(call)                                  \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_code(e_); \
    } while (0)

// Q_p^T (trans = 1) or Q_p (trans = 0) of panel p on k columns; Bsrc/ldbs
// address the panel's first row of the input, B/ldb of the output.
inline bool is_mixed(const tsqr_factors_s *f) { return f->plan.opts.prec == TSQR_MIXED; }

// Leaf part of Q_p^T / Q_p: FP64 reflectors, or the FP32 copy in the mixed mode.
hipError_t leaf_apply(const tsqr_factors_s *f, const Panel &p, const double *Bsrc, int64_t ldbs, double *B,
                      int64_t ldb, int64_t k, int trans, hipStream_t st) {
    const Plan &P = f->plan;
    const PanelArgs pa = panel_args(p, f->ws);
    const int64_t off = p.row_off + (int64_t)p.col_off * P.m;
    const double *Tc = at<double>(f, p.off_tc);
    if (k <= tsqr::kApply3MaxCols && Bsrc == B && p.off_pz) {
        // few columns: chunk-parallel three-pass form
        double *Pc = at<double>(f, p.off_pz);
        double *Zc = Pc + (size_t)p.n * 16 * (size_t)p.total_chunks;
        if (is_mixed(f))
            return tsqr::launch_leaf_apply3_32(at<float>(f, P.off_w32) + off, P.m, Tc, pa, B, ldb, k, trans, Pc,
                                               Zc, st);
        return tsqr::launch_leaf_apply3(at<double>(f, P.off_w) + off, P.m, Tc, pa, B, ldb, k, trans, Pc, Zc,
                                        st);
    }
    if (is_mixed(f))
        return tsqr::launch_leaf_apply_m32(at<float>(f, P.off_w32) + off, P.m, Tc, pa, Bsrc, ldbs, B, ldb,
                                           k, trans, st);
    return tsqr::launch_leaf_apply_m(at<double>(f, P.off_w) + off, P.m, Tc, pa, Bsrc, ldbs, B, ldb, k,
                                     trans, st);
}

int panel_apply(const tsqr_factors_s *f, const Panel &p, const double *Bsrc, int64_t ldbs, double *B,
                int64_t ldb, int64_t k, int trans, hipStream_t st) {
    const PanelArgs pa = panel_args(p, f->ws);
    const double *Rdom = at<double>(f, p.off_rdom);
    const double *Tnode = at<double>(f, p.off_tnode);
    auto levels = tsqr::tree_levels(p.P, p.tree);
    if (trans) {
        TRY(leaf_apply(f, p, Bsrc, ldbs, B, ldb, k, 1, st));
        for (const auto &L : levels) {
            TreeArgs ta{L.stride, L.span, L.chains, L.width};
            TRY(tsqr::launch_tree_apply(Rdom, Tnode, pa, ta, B, ldb, k, 1, st));
        }
    } else {
        if (Bsrc != B) TRY(tsqr::launch_copy(Bsrc, ldbs, B, ldb, p.m, k, st));
        for (auto it = levels.rbegin(); it != levels.rend(); ++it) {
            TreeArgs ta{it->stride, it->span, it->chains, it->width};
            TRY(tsqr::launch_tree_apply(Rdom, Tnode, pa, ta, B, ldb, k, 0, st));
        }
        TRY(leaf_apply(f, p, B, ldb, B, ldb, k, 0, st));
    }
    return 0;
}

int validate_handle(const tsqr_factors_s *f, bool need_q) {
    if (!f) return -1;
    if (need_q && !f->keep_q) return TSQR_ERR_STATE;
    return 0;
}

}  // namespace

extern "C" {

TSQR_API void tsqr_default_opts(tsqr_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->row_block = 0;
    o->tree = TSQR_TREE_BINARY;
    o->prec = TSQR_F64;
    o->keep_q = 1;
    o->lsq_max_rhs = 8;
    o->refine_max_iter = 30;
    o->refine_tol = 1e-14;
}

TSQR_API size_t tsqr_workspace_bytes(int64_t m, int64_t n, const tsqr_opts *o) {
    Plan p;
    if (tsqr::make_plan(m, n, o, &p) != 0) return 0;
    return p.total;
}

TSQR_API int64_t tsqr_partition(int64_t m, int64_t n, const tsqr_opts *o, int64_t *row0, int64_t *nrows,
                                int64_t cap) {
    Plan p;
    int rc = tsqr::make_plan(m, n, o, &p);
    if (rc) return rc;
    const Panel &pa = p.panels[0];
    for (int64_t i = 0; i < pa.P && i < cap; ++i) {
        if (row0) row0[i] = pa.domain_row0(i);
        if (nrows) nrows[i] = pa.domain_rows(i);
    }
    return pa.P;
}

TSQR_API int tsqr_plan_info(int64_t m, int64_t n, const tsqr_opts *o, int64_t *num_domains,
                            int64_t *chunk_rows, int64_t *num_panels) {
    Plan p;
    int rc = tsqr::make_plan(m, n, o, &p);
    if (rc) return rc;
    if (num_domains) *num_domains = p.panels[0].P;
    if (chunk_rows) *chunk_rows = p.panels[0].chunk;
    if (num_panels) *num_panels = (int64_t)p.panels.size();
    return 0;
}

}  // extern "C"

static int factor_enqueue(tsqr_factors_s *f, const double *A, int64_t lda, hipStream_t st);

// tsqr_factor into a caller-provided handle (which this call fills in);
// the handle's owner frees nothing here.
int tsqr::factor_into(tsqr_factors_s *f, int64_t m, int64_t n, const double *A, int64_t lda,
                      const tsqr_opts *o, void *dwork, size_t work_bytes, hipStream_t st) {
    tsqr_opts defaults;
    tsqr_default_opts(&defaults);
    if (!o) o = &defaults;
    Plan plan;
    int rc = tsqr::make_plan(m, n, o, &plan);
    if (rc) return rc;
    if (!A) return -3;
    if (lda < m) return -4;
    if (!dwork || work_bytes < plan.total || (reinterpret_cast<uintptr_t>(dwork) % tsqr::kAlign))
        return TSQR_ERR_WORKSPACE;
    f->plan = plan;
    f->ws = static_cast<char *>(dwork);
    f->ws_bytes = work_bytes;
    f->keep_q = o->keep_q ? 1 : 0;
    f->last_refine = 0;
    f->last_k = 0;
    f->route_checked = 0;
    f->kappa_est = 0.0;
    return factor_enqueue(f, A, lda, st);
}

extern "C" {

TSQR_API int tsqr_factor(int64_t m, int64_t n, const double *A, int64_t lda, const tsqr_opts *o,
                         void *dwork, size_t work_bytes, void *stream, tsqr_factors *out) {
    if (!out) return -9;
    *out = nullptr;
    tsqr_factors_s *f = new (std::nothrow) tsqr_factors_s;
    if (!f) return TSQR_ERR_WORKSPACE;
    const int rc = tsqr::factor_into(f, m, n, A, lda, o, dwork, work_bytes, static_cast<hipStream_t>(stream));
    if (rc) {
        delete f;
        return rc;
    }
    *out = f;
    return 0;
}

}  // extern "C"

// The kernels of a factorization whose handle is filled in (plan, workspace).
static int factor_enqueue(tsqr_factors_s *f, const double *A, int64_t lda, hipStream_t st) {
    const Plan &plan = f->plan;
    const int64_t m = plan.m, n = plan.n;
    double *W = at<double>(f, plan.off_w);
    double *R = at<double>(f, plan.off_r);
    double *dsign = at<double>(f, plan.off_d);
    const int np = (int)plan.panels.size();
    int err = 0;
    if (np > 1) {
        // the panels write R block by block; its lower-left part stays zero
        hipError_t e = tsqr::launch_fill(R, n * n, 0.0, st);
        if (e != hipSuccess) err = hip_code(e);
    }
    for (int q = 0; q < np && !err; ++q) {
        const Panel &p = plan.panels[q];
        const PanelArgs pa = panel_args(p, f->ws);
        if (!p.wchunk0.empty()) {
            // the weighted partition's table, for this and every later call
            // on the factor (copied from host memory before the call returns)
            hipError_t e = hipMemcpyAsync(f->ws + p.off_wtab, p.wchunk0.data(), sizeof(int64_t) * p.wchunk0.size(),
                                          hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                err = hip_code(e);
                break;
            }
        }
        const double *src = (q == 0) ? A : W;
        const int64_t lds = (q == 0) ? lda : m;
        const double *src_p = src + p.row_off + (int64_t)p.col_off * lds;
        double *V = W + p.row_off + (int64_t)p.col_off * m;
        const int keep = (f->keep_q || q < np - 1) ? 1 : 0;
        double *Rdom = at<double>(f, p.off_rdom);
        double *Tnode = at<double>(f, p.off_tnode);
        double *Tc = at<double>(f, p.off_tc);
        hipError_t e =
            (plan.opts.prec == TSQR_MIXED)
                ? tsqr::launch_leaf32(src_p, lds, at<float>(f, plan.off_w32) + (V - W), m, Tc, Rdom, pa, keep, st)
                : tsqr::launch_leaf(src_p, lds, V, m, Tc, Rdom, pa, keep, st);
        for (const auto &L : tsqr::tree_levels(p.P, p.tree)) {
            if (e != hipSuccess) break;
            TreeArgs ta{L.stride, L.span, L.chains, L.width};
            e = tsqr::launch_tree_level(Rdom, Tnode, pa, ta, keep, st);
        }
        if (e == hipSuccess && keep) e = tsqr::launch_tree_t(Tnode, pa, st);
        if (e == hipSuccess)
            e = tsqr::launch_sign_normalise(Rdom, p.n, R, n, p.row_off, p.col_off, dsign, st);
        if (e != hipSuccess) {
            err = hip_code(e);
            break;
        }
        if (q < np - 1) {
            // trailing update: Q_p^T on columns [col_off + w, n), rows [row_off, m)
            const int64_t c1 = p.col_off + p.n;
            const int64_t kt = n - c1;
            const double *bsrc = src + p.row_off + c1 * lds;
            double *bdst = W + p.row_off + c1 * m;
            err = panel_apply(f, p, bsrc, lds, bdst, m, kt, 1, st);
            if (err) break;
            // R[row_off : row_off + w, c1 : n] = D_p * (top w rows of the result)
            e = tsqr::launch_copy(bdst, m, R + p.row_off + c1 * n, n, p.n, kt, st);
            if (e == hipSuccess) e = tsqr::launch_scale_rows(R + p.row_off + c1 * n, n, p.n, kt,
                                                            dsign + p.row_off, st);
            if (e != hipSuccess) err = hip_code(e);
        }
    }
    return err;
}

extern "C" {

TSQR_API int tsqr_get_r(tsqr_factors f, double *R, int64_t ldr, void *stream) {
    int rc = validate_handle(f, false);
    if (rc) return rc;
    if (!R) return -2;
    if (ldr < f->plan.n) return -3;
    hipError_t e = tsqr::launch_copy(at<double>(f, f->plan.off_r), f->plan.n, R, ldr, f->plan.n,
                                     f->plan.n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : hip_code(e);
}

TSQR_API int tsqr_apply_qt(tsqr_factors f, int64_t k, double *B, int64_t ldb, void *stream) {
    int rc = validate_handle(f, true);
    if (rc) return rc;
    if (k < 0) return -2;
    if (k == 0) return 0;
    if (!B) return -3;
    if (ldb < f->plan.m) return -4;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double *d = at<double>(f, f->plan.off_d);
    for (const Panel &p : f->plan.panels) {
        double *Bp = B + p.row_off;
        rc = panel_apply(f, p, Bp, ldb, Bp, ldb, k, 1, st);
        if (rc) return rc;
        hipError_t e = tsqr::launch_scale_rows(Bp, ldb, p.n, k, d + p.row_off, st);
        if (e != hipSuccess) return hip_code(e);
    }
    return 0;
}

static int apply_q_impl(tsqr_factors_s *f, int64_t k, double *B, int64_t ldb, bool scale,
                        bool skip_left_cols, hipStream_t st) {
    const double *d = at<double>(f, f->plan.off_d);
    if (scale)
        for (const Panel &p : f->plan.panels) {
            hipError_t e = tsqr::launch_scale_rows(B + p.row_off, ldb, p.n, k, d + p.row_off, st);
            if (e != hipSuccess) return hip_code(e);
        }
    for (auto it = f->plan.panels.rbegin(); it != f->plan.panels.rend(); ++it) {
        const Panel &p = *it;
        const int64_t c0 = skip_left_cols ? p.col_off : 0;
        double *Bp = B + p.row_off + c0 * ldb;
        int rc = panel_apply(f, p, Bp, ldb, Bp, ldb, k - c0, 0, st);
        if (rc) return rc;
    }
    return 0;
}

// Backward-error bounds of the last mixed solve (lsq_max_rhs doubles in the
// refinement scratch, after the partial sums and the sweep history).
static double *mixed_eta(const tsqr_factors_s *f) {
    const Plan &P = f->plan;
    const int kmax = P.opts.lsq_max_rhs < 8 ? P.opts.lsq_max_rhs : 8;
    double *Xw = at<double>(f, P.off_ref);
    return Xw + (size_t)P.n * kmax + (size_t)tsqr::kRefineBlocks * P.n * kmax +
           (size_t)tsqr::kRefineBlocks * 2 * kmax + 2 * (size_t)kmax;
}

// Mixed-precision least squares: Bjorck refinement of the augmented system
// [I A; A^T 0][r; x] = [b; 0] from r = 0, x = 0, so the first sweep is the
// plain solve through the mixed factor.  Per sweep (groups of at most 8
// right-hand sides):
//   f = b - r - A x, g = -A^T r          (FP64, one pass over A)
//   F = Q^T f                            (FP32 leaves, FP64 tree)
//   R^T h = g, dx = R^{-1}(F[0:n] - h), x += dx, F[0:n] = h
//   r += Q F                             (skipped after the last sweep)
// The stream is synchronised once per sweep to read the convergence flag.
static int lsq_solve_mixed(tsqr_factors_s *f, const double *A, int64_t lda, int64_t k, const double *B,
                           int64_t ldb, double *X, int64_t ldx, double *resid, int32_t *dinfo,
                           hipStream_t st) {
    const Plan &P = f->plan;
    const int n = (int)P.n;
    const int64_t m = P.m;
    const int kmax = P.opts.lsq_max_rhs < 8 ? P.opts.lsq_max_rhs : 8;
    const int nb = tsqr::resid_blocks(m);
    double *F = at<double>(f, P.off_lsq);
    double *Rr = at<double>(f, P.off_lsq2);
    double *Xw = at<double>(f, P.off_ref);
    double *gpart = Xw + (size_t)n * kmax;
    double *rpart = gpart + (size_t)tsqr::kRefineBlocks * n * kmax;
    double *hist = rpart + (size_t)tsqr::kRefineBlocks * 2 * kmax;   // rel (kmax), ||g|| (kmax)
    double *eta = mixed_eta(f);
    int32_t *status = reinterpret_cast<int32_t *>(eta + P.opts.lsq_max_rhs);
    const double *Rf = at<double>(f, P.off_r);
    int sweeps_max = 0;
    for (int64_t c0 = 0; c0 < k; c0 += kmax) {
        const int kg = (int)((k - c0 < kmax) ? k - c0 : kmax);
        const double *Bg = B + c0 * ldb;
        TRY(tsqr::launch_fill(Xw, (int64_t)n * kg, 0.0, st));
        TRY(tsqr::launch_fill(Rr, m * kg, 0.0, st));
        TRY(tsqr::launch_status_init(status, hist, kg, st));
        int sweeps = 0;
        for (int it = 0; it <= P.opts.refine_max_iter; ++it) {
            TRY(tsqr::launch_lsq_resid(A, lda, m, n, Bg, ldb, Xw, n, Rr, F, kg, gpart, rpart, nb, st));
            int rc = tsqr_apply_qt(f, kg, F, m, st);
            if (rc) return rc;
            TRY(tsqr::launch_lsq_refine(Rf, n, F, m, kg, gpart, nb, Xw, n, P.opts.refine_tol, status, hist,
                                        hist + kmax, st));
            int32_t hs[2] = {0, 0};
            TRY(hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, st));
            TRY(hipStreamSynchronize(st));
            sweeps = hs[0];
            if (hs[1] || it == P.opts.refine_max_iter) break;
            rc = apply_q_impl(f, kg, F, m, true, false, st);
            if (rc) return rc;
            TRY(tsqr::launch_axpy(Rr, F, m * kg, st));
        }
        if (sweeps > sweeps_max) sweeps_max = sweeps;
        TRY(tsqr::launch_mixed_final(Rf, n, kg, Xw, X + c0 * ldx, ldx, resid ? resid + c0 : nullptr, dinfo,
                                     c0 > 0 ? 1 : 0, rpart, nb, hist + kmax, eta + c0, st));
    }
    f->last_refine = sweeps_max;
    f->last_k = k;
    return 0;
}

TSQR_API int tsqr_apply_q(tsqr_factors f, int64_t k, double *B, int64_t ldb, void *stream) {
    int rc = validate_handle(f, true);
    if (rc) return rc;
    if (k < 0) return -2;
    if (k == 0) return 0;
    if (!B) return -3;
    if (ldb < f->plan.m) return -4;
    return apply_q_impl(f, k, B, ldb, true, false, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Thin Q of a single-panel FP64 factor: the top-down tree on n x n blocks,
// then the MFMA leaf; `before_leaf`, if set, is an event the leaf waits for.
static int form_q_single_panel(tsqr_factors_s *f, double *Q, int64_t ldq, hipStream_t st,
                               hipEvent_t before_leaf) {
    const double *dsign = at<double>(f, f->plan.off_d);
    {
        const Panel &p = f->plan.panels[0];
        const PanelArgs pa = panel_args(p, f->ws);
        double *S = at<double>(f, p.off_s);
        const auto levels = tsqr::tree_levels(p.P, p.tree);
        const int nlev = (int)levels.size();
        // the top levels in one launch, one workgroup per path to a left of
        // level lstop - 1 (at most kTopPaths of them); the rest level by level
        constexpr int64_t kTopPaths = 32;
        // (the path walk assumes one left per span: not for the XCD tree)
        int lstop = nlev;
        for (int L = 0; L < nlev && p.tree != TSQR_TREE_XCD; ++L)
            if ((p.P + levels[L].stride - 1) / levels[L].stride <= kTopPaths) {
                lstop = L;
                break;
            }
        if (lstop < nlev && nlev <= tsqr::kMaxTreeLevels) {
            tsqr::TreePath tp{};
            tp.nlev = nlev;
            for (int L = 0; L < nlev; ++L) {
                tp.stride[L] = levels[L].stride;
                tp.span[L] = levels[L].span;
            }
            TRY(tsqr::launch_tree_down_top(at<double>(f, p.off_rdom), at<double>(f, p.off_tnode), dsign, S, pa,
                                           tp, lstop, levels[lstop].stride, st));
        } else {
            lstop = nlev;
            TRY(tsqr::launch_seed_root(S, p.n, dsign, st));
        }
        for (int L = lstop - 1; L >= 0; --L) {
            TreeArgs ta{levels[L].stride, levels[L].span, levels[L].chains, levels[L].width};
            TRY(tsqr::launch_tree_down(at<double>(f, p.off_rdom), at<double>(f, p.off_tnode), S, pa, ta,
                                       st));
        }
        if (before_leaf) TRY(hipStreamWaitEvent(st, before_leaf, 0));
        TRY(tsqr::launch_form_leaf(at<double>(f, f->plan.off_w), f->plan.m, at<double>(f, p.off_tc), S,
                                   pa, Q, ldq, st));
    }
    return 0;
}

extern "C" {

TSQR_API int tsqr_form_q(tsqr_factors f, double *Q, int64_t ldq, void *stream) {
    int rc = validate_handle(f, true);
    if (rc) return rc;
    if (!Q) return -2;
    if (ldq < f->plan.m) return -3;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (f->plan.panels.size() == 1 && !is_mixed(f)) return form_q_single_panel(f, Q, ldq, st, nullptr);
    const double *dsign = at<double>(f, f->plan.off_d);
    hipError_t e = tsqr::launch_fill_identity_signs(Q, ldq, f->plan.m, (int)f->plan.n, dsign, st);
    if (e != hipSuccess) return hip_code(e);
    return apply_q_impl(f, f->plan.n, Q, ldq, false, true, st);
}

namespace {

// TSLU's workspace: the candidate rows of every domain (P x b, int32) and a
// 64 x 64 block for L11.
size_t tslu_up(size_t x) { return (x + tsqr::kAlign - 1) / tsqr::kAlign * tsqr::kAlign; }

// TSLU's workspace: the candidate rows of every domain (P x b, int32), a
// 64 x 64 block for L11 and a weighted partition's table.
size_t tslu_bytes(const Plan &p, int64_t b) {
    const Panel &pp = p.panels[0];
    return tslu_up((size_t)pp.P * (size_t)b * sizeof(int32_t)) + tslu_up(sizeof(double) * 64 * 64) +
           sizeof(int64_t) * pp.wchunk0.size();
}

}  // namespace

TSQR_API size_t tsqr_tslu_workspace_bytes(int64_t m, int64_t b, const tsqr_opts *o) {
    if (b < 1 || b > tsqr::kMaxPanel) return 0;
    Plan p;
    if (tsqr::make_plan(m, b, o, &p) != 0) return 0;
    return tslu_bytes(p, b);
}

TSQR_API int tsqr_tslu(int64_t m, int64_t b, const double *A, int64_t lda, const tsqr_opts *o, void *dwork,
                       size_t work_bytes, double *L, int64_t ldl, double *U, int64_t ldu, int64_t *ipiv,
                       int32_t *dinfo, void *stream) {
    if (b > tsqr::kMaxPanel) return TSQR_ERR_UNSUPPORTED;
    if (b < 1) return -2;
    Plan p;
    const int rc = tsqr::make_plan(m, b, o, &p);
    if (rc) return rc;
    if (!A) return -3;
    if (lda < m) return -4;
    if (!L || ldl < m) return -6;
    if (!U || ldu < b) return -7;
    if (!ipiv) return -8;
    const size_t need = tslu_bytes(p, b);
    if (!dwork || work_bytes < need || (reinterpret_cast<uintptr_t>(dwork) % tsqr::kAlign))
        return TSQR_ERR_WORKSPACE;
    const Panel &pp = p.panels[0];
    std::vector<TreeArgs> levels;
    for (const auto &Lv : tsqr::tree_levels(pp.P, pp.tree)) levels.push_back(TreeArgs{Lv.stride, Lv.span, Lv.chains, Lv.width});
    char *w = static_cast<char *>(dwork);
    int32_t *cand = reinterpret_cast<int32_t *>(w);
    const size_t off_l11 = tslu_up((size_t)pp.P * (size_t)b * sizeof(int32_t));
    double *L11 = reinterpret_cast<double *>(w + off_l11);
    PanelArgs pa = panel_args(pp);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!pp.wchunk0.empty()) {
        int64_t *tab = reinterpret_cast<int64_t *>(w + off_l11 + tslu_up(sizeof(double) * 64 * 64));
        hipError_t e = hipMemcpyAsync(tab, pp.wchunk0.data(), sizeof(int64_t) * pp.wchunk0.size(),
                                      hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_code(e);
        pa.wtab = tab;
    }
    hipError_t e = tsqr::launch_tslu(A, lda, pa, levels, (int)b, cand, L11, L, ldl, U, ldu, ipiv, dinfo, st);
    return e == hipSuccess ? 0 : hip_code(e);
}

TSQR_API int tsqr_cholesky(int64_t n, double *A, int64_t lda, int32_t *dinfo, void *stream) {
    if (n < 0) return -1;
    if (n > INT32_MAX) return TSQR_ERR_UNSUPPORTED;
    if (!A && n > 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (!dinfo) return -4;
    hipError_t e = tsqr::launch_cholesky(n, A, lda, dinfo, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : hip_code(e);
}

namespace {

// CALU's workspace: the TSLU workspace of the panel that needs the most,
// then L (m x 64), U (64 x 64), the pivot rows (64 int64), the interchange
// record (kCaluMetaWords int32) and the panel's info word.
struct CaluLayout {
    size_t tslu = 0, l = 0, u = 0, piv = 0, swp = 0, pinfo = 0, total = 0;
};
int calu_layout(int64_t m, int64_t n, const tsqr_opts *o, CaluLayout *out) {
    // the TSLU workspace of the panel that needs the most (every panel's
    // plan is made again when it is factored)
    size_t tsb = 0;
    for (int64_t k = 0; k < n; k += 64) {
        const int64_t b = n - k < 64 ? n - k : 64;
        Plan p;
        const int rc = tsqr::make_plan(m - k, b, o, &p);
        if (rc) return rc;
        if (!p.panels[0].wchunk0.empty()) return TSQR_ERR_UNSUPPORTED;
        tsb = std::max(tsb, tslu_bytes(p, b));
    }
    CaluLayout L;
    L.tslu = 0;
    L.l = tslu_up(tsb);
    L.u = L.l + tslu_up(sizeof(double) * (size_t)m * 64);
    L.piv = L.u + tslu_up(sizeof(double) * 64 * 64);
    L.swp = L.piv + tslu_up(sizeof(int64_t) * 64);
    L.pinfo = L.swp + tslu_up(sizeof(int32_t) * tsqr::kCaluMetaWords);
    L.total = L.pinfo + tslu_up(sizeof(int32_t));
    *out = L;
    return 0;
}

}  // namespace

TSQR_API size_t tsqr_calu_workspace_bytes(int64_t m, int64_t n, const tsqr_opts *o) {
    if (n < 1 || m < n) return 0;
    CaluLayout L;
    if (calu_layout(m, n, o, &L) != 0) return 0;
    return L.total;
}

TSQR_API int tsqr_calu(int64_t m, int64_t n, double *A, int64_t lda, const tsqr_opts *o, void *dwork,
                       size_t work_bytes, int64_t *ipiv, int32_t *dinfo, void *stream) {
    if (n < 1) return -2;
    if (m < n) return -1;
    if (m > INT32_MAX) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -3;
    if (lda < m) return -4;
    CaluLayout Lw;
    const int rc = calu_layout(m, n, o, &Lw);
    if (rc) return rc;
    if (!ipiv) return -8;
    if (!dinfo) return -9;
    if (!dwork || work_bytes < Lw.total || (reinterpret_cast<uintptr_t>(dwork) % tsqr::kAlign))
        return TSQR_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(dwork);
    double *Lp = reinterpret_cast<double *>(w + Lw.l);
    double *Up = reinterpret_cast<double *>(w + Lw.u);
    int64_t *piv = reinterpret_cast<int64_t *>(w + Lw.piv);
    int32_t *swp = reinterpret_cast<int32_t *>(w + Lw.swp);
    int32_t *pinfo = reinterpret_cast<int32_t *>(w + Lw.pinfo);
    hipError_t e = tsqr::launch_calu_clear(dinfo, st);
    if (e != hipSuccess) return hip_code(e);
    for (int64_t k = 0; k < n; k += 64) {
        const int b = (int)(n - k < 64 ? n - k : 64);
        const int64_t mr = m - k;
        Plan p;
        const int prc = tsqr::make_plan(mr, b, o, &p);
        if (prc) return prc;
        const Panel &pp = p.panels[0];
        std::vector<TreeArgs> levels;
        for (const auto &Lv : tsqr::tree_levels(pp.P, pp.tree))
            levels.push_back(TreeArgs{Lv.stride, Lv.span, Lv.chains, Lv.width});
        int32_t *cand = reinterpret_cast<int32_t *>(w);
        double *L11 = reinterpret_cast<double *>(w + tslu_up((size_t)pp.P * (size_t)b * sizeof(int32_t)));
        double *Ak = A + k + k * lda;
        e = tsqr::launch_tslu(Ak, lda, panel_args(pp), levels, b, cand, L11, Lp, mr, Up, 64, piv, pinfo, st);
        if (e != hipSuccess) return hip_code(e);
        e = tsqr::launch_calu_panel_rest(A, lda, m, n, k, b, piv, swp, ipiv, pinfo, dinfo, Lp, mr, Up, 64, st);
        if (e != hipSuccess) return hip_code(e);
    }
    return 0;
}

TSQR_API int tsqr_cond_estimate(tsqr_factors f, double *kappa, void *stream) {
    int rc = validate_handle(f, false);
    if (rc) return rc;
    if (!kappa) return -2;
    if (f->plan.n > tsqr::kMaxMixedN) return TSQR_ERR_UNSUPPORTED;
    hipError_t e = tsqr::launch_cond_est(at<double>(f, f->plan.off_r), (int)f->plan.n, kappa,
                                         static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : hip_code(e);
}

TSQR_API int tsqr_route_info(tsqr_factors f, int32_t *prec, double *kappa_est) {
    int rc = validate_handle(f, false);
    if (rc) return rc;
    if (prec) *prec = f->plan.opts.prec;
    if (kappa_est) *kappa_est = f->kappa_est;
    return 0;
}

}  // extern "C"

// Mixed-precision routing (opts.route_kappa): at the first solve of a mixed
// factor, estimate kappa_1(R) (for n <= 64 R is exact to FP64 rounding, for
// wider matrices to FP32 rounding, plenty for an estimate); above the
// threshold, or not finite, factor A again in FP64 into the same workspace
// (the FP64 plan is the mixed one without its FP32 reflectors and refinement
// scratch, so it fits) and the handle becomes an FP64 factor.
static int route_mixed(tsqr_factors_s *f, const double *A, int64_t lda, hipStream_t st, bool *routed) {
    *routed = false;
    const Plan &P = f->plan;
    if (!(P.opts.route_kappa > 0.0) || f->route_checked) return 0;
    f->route_checked = 1;
    double *kd = at<double>(f, P.off_cond);
    TRY(tsqr::launch_cond_est(at<double>(f, P.off_r), (int)P.n, kd, st));
    double kh = 0.0;
    TRY(hipMemcpyAsync(&kh, kd, sizeof(double), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    f->kappa_est = kh;
    if (kh <= P.opts.route_kappa) return 0;
    tsqr_opts o = P.opts;
    o.prec = TSQR_F64;
    Plan p64;
    if (tsqr::make_plan(P.m, P.n, &o, &p64) != 0 || p64.total > f->ws_bytes) return 0;
    f->plan = p64;
    const int rc = factor_enqueue(f, A, lda, st);
    if (rc) return rc;
    *routed = true;
    return 0;
}

extern "C" {

TSQR_API int tsqr_lsq_solve(tsqr_factors f, const double *A, int64_t lda, int64_t k, const double *B,
                            int64_t ldb, double *X, int64_t ldx, double *resid, int32_t *dinfo,
                            void *stream) {
    int rc = validate_handle(f, true);
    if (rc) return rc;
    const Plan &P = f->plan;
    if (P.opts.prec == TSQR_MIXED && !A) return -2;
    if (A && lda < P.m) return -3;
    if (k < 1 || k > P.opts.lsq_max_rhs) return -4;
    if (!B) return -5;
    if (ldb < P.m) return -6;
    if (!X) return -7;
    if (ldx < P.n) return -8;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (P.opts.prec == TSQR_MIXED) {
        bool routed = false;
        rc = route_mixed(f, A, lda, st, &routed);
        if (rc) return rc;
        if (!routed) return lsq_solve_mixed(f, A, lda, k, B, ldb, X, ldx, resid, dinfo, st);
    }
    double *C = at<double>(f, P.off_lsq);
    hipError_t e = tsqr::launch_copy(B, ldb, C, P.m, P.m, k, st);
    if (e != hipSuccess) return hip_code(e);
    rc = tsqr_apply_qt(f, k, C, P.m, stream);
    if (rc) return rc;
    e = tsqr::launch_lsq_finish(at<double>(f, P.off_r), (int)P.n, C, P.m, P.m, k, X, ldx, resid, dinfo,
                                at<double>(f, P.off_small), st);
    f->last_refine = 0;
    return e == hipSuccess ? 0 : hip_code(e);
}

}  // extern "C"

namespace {

// tsqr_factor_solve's second stream and its three events, per device,
// created on first use and kept until the process ends.  g_fork_mu is held
// while a call enqueues its work, so the events' record/wait pairs of two
// concurrent calls do not interleave.
struct ForkJoin {
    hipStream_t aux = nullptr;
    hipEvent_t leaf = nullptr, tree = nullptr, done = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_fork_mu;
ForkJoin g_fork[kMaxDevices];

int fork_join_for_current_device(ForkJoin **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_code(e);
    if (dev < 0 || dev >= kMaxDevices) return TSQR_ERR_UNSUPPORTED;
    ForkJoin &fj = g_fork[dev];
    if (!fj.aux) {
        ForkJoin n;
        e = hipStreamCreateWithFlags(&n.aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.leaf, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.tree, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_code(e);
        fj = n;
    }
    *out = &fj;
    return 0;
}

// The fork/join schedule of tsqr_factor_solve for a single-panel FP64
// factor (caller holds g_fork_mu).  main: leaf, tree, signs, thin Q.  aux:
// after the leaf, the chunks' T factors and the solve's copy and leaf pass
// of Q^T B; after the tree, its tree pass and the triangular solve.  main
// finally waits for aux.
int factor_solve_forked(tsqr_factors_s *f, const double *A, int64_t lda, int64_t k, const double *B,
                        int64_t ldb, double *X, int64_t ldx, double *resid, int32_t *dinfo, double *Q,
                        int64_t ldq, hipStream_t st, const ForkJoin &fj) {
    const Plan &P = f->plan;
    const Panel &p = P.panels[0];
    const PanelArgs pa = panel_args(p, f->ws);
    double *W = at<double>(f, P.off_w);
    double *Rdom = at<double>(f, p.off_rdom);
    double *Tnode = at<double>(f, p.off_tnode);
    double *C = at<double>(f, P.off_lsq);
    const auto levels = tsqr::tree_levels(p.P, p.tree);
    double *Tc = at<double>(f, p.off_tc);
    if (!p.wchunk0.empty())
        TRY(hipMemcpyAsync(f->ws + p.off_wtab, p.wchunk0.data(), sizeof(int64_t) * p.wchunk0.size(),
                           hipMemcpyHostToDevice, st));
    TRY(tsqr::launch_leaf(A, lda, W, P.m, Tc, Rdom, pa, 2, st));
    TRY(hipEventRecord(fj.leaf, st));
    TRY(hipStreamWaitEvent(fj.aux, fj.leaf, 0));
    // the chunks' T factors (the leaf stored their Gram entries), beside the
    // tree: the tree does not read them; the solve's leaf pass and the thin
    // Q's leaf kernel (after fj.done) do
    TRY(tsqr::launch_chunk_t(Tc, pa, p.total_chunks, fj.aux));
    TRY(tsqr::launch_copy(B, ldb, C, P.m, P.m, k, fj.aux));
    TRY(leaf_apply(f, p, C, P.m, C, P.m, k, 1, fj.aux));
    for (const auto &L : levels) {
        TreeArgs ta{L.stride, L.span, L.chains, L.width};
        TRY(tsqr::launch_tree_level(Rdom, Tnode, pa, ta, 1, st));
    }
    TRY(tsqr::launch_tree_t(Tnode, pa, st));
    TRY(tsqr::launch_sign_normalise(Rdom, p.n, at<double>(f, P.off_r), P.n, p.row_off, p.col_off,
                                    at<double>(f, P.off_d), st));
    TRY(hipEventRecord(fj.tree, st));
    TRY(hipStreamWaitEvent(fj.aux, fj.tree, 0));
    for (const auto &L : levels) {
        TreeArgs ta{L.stride, L.span, L.chains, L.width};
        TRY(tsqr::launch_tree_apply(Rdom, Tnode, pa, ta, C, P.m, k, 1, fj.aux));
    }
    // rows 0..n-1 of Q^T B for the sign-normalised Q (as tsqr_apply_qt)
    TRY(tsqr::launch_scale_rows(C + p.row_off, P.m, p.n, k, at<double>(f, P.off_d) + p.row_off, fj.aux));
    TRY(tsqr::launch_lsq_finish(at<double>(f, P.off_r), (int)P.n, C, P.m, P.m, k, X, ldx, resid, dinfo,
                                at<double>(f, P.off_small), fj.aux));
    TRY(hipEventRecord(fj.done, fj.aux));
    // the thin Q's top-down tree runs beside the solve's tree pass; its leaf
    // kernel (which fills the GPU) starts once the solve is done
    if (Q) {
        const int rc = form_q_single_panel(f, Q, ldq, st, fj.done);
        if (rc) {
            (void)hipStreamWaitEvent(st, fj.done, 0);
            return rc;
        }
        return 0;
    }
    const hipError_t e = hipStreamWaitEvent(st, fj.done, 0);
    return e == hipSuccess ? 0 : hip_code(e);
}

}  // namespace

extern "C" {

TSQR_API int tsqr_factor_solve(int64_t m, int64_t n, const double *A, int64_t lda, const tsqr_opts *o,
                               void *dwork, size_t work_bytes, int64_t k, const double *B, int64_t ldb,
                               double *X, int64_t ldx, double *resid, int32_t *dinfo, double *Q,
                               int64_t ldq, void *stream, tsqr_factors *out) {
    if (!out) return -18;
    *out = nullptr;
    tsqr_opts defaults;
    tsqr_default_opts(&defaults);
    if (!o) o = &defaults;
    Plan plan;
    int rc = tsqr::make_plan(m, n, o, &plan);
    if (rc) return rc;
    if (!A) return -3;
    if (lda < m) return -4;
    if (!o->keep_q) return TSQR_ERR_STATE;
    if (!dwork || work_bytes < plan.total || (reinterpret_cast<uintptr_t>(dwork) % tsqr::kAlign))
        return TSQR_ERR_WORKSPACE;
    if (k < 1 || k > o->lsq_max_rhs) return -8;
    if (!B) return -9;
    if (ldb < m) return -10;
    if (!X) return -11;
    if (ldx < n) return -12;
    if (Q && ldq < m) return -16;
    if (o->prec != TSQR_F64 || plan.panels.size() != 1) {
        // the three calls in order on `stream`
        rc = tsqr_factor(m, n, A, lda, o, dwork, work_bytes, stream, out);
        if (rc) return rc;
        rc = tsqr_lsq_solve(*out, A, lda, k, B, ldb, X, ldx, resid, dinfo, stream);
        if (!rc && Q) rc = tsqr_form_q(*out, Q, ldq, stream);
        if (rc) {
            tsqr_free(*out);
            *out = nullptr;
        }
        return rc;
    }
    tsqr_factors_s *f = new (std::nothrow) tsqr_factors_s;
    if (!f) return TSQR_ERR_WORKSPACE;
    f->plan = plan;
    f->ws = static_cast<char *>(dwork);
    f->ws_bytes = work_bytes;
    f->keep_q = 1;
    f->last_refine = 0;
    {
        std::lock_guard<std::mutex> lock(g_fork_mu);
        ForkJoin *fj = nullptr;
        rc = fork_join_for_current_device(&fj);
        if (!rc) rc = factor_solve_forked(f, A, lda, k, B, ldb, X, ldx, resid, dinfo, Q, ldq,
                                          static_cast<hipStream_t>(stream), *fj);
    }
    if (rc) {
        delete f;
        return rc;
    }
    *out = f;
    return 0;
}

TSQR_API int tsqr_lsq_backward_error(tsqr_factors f, int64_t k, double *eta, void *stream) {
    int rc = validate_handle(f, true);
    if (rc) return rc;
    if (!is_mixed(f) || !f->last_k) return TSQR_ERR_STATE;
    if (k < 1 || k > f->last_k) return -2;
    if (!eta) return -3;
    const hipError_t e = hipMemcpyAsync(eta, mixed_eta(f), sizeof(double) * (size_t)k, hipMemcpyDeviceToDevice,
                                        static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : hip_code(e);
}

static size_t orth_align(size_t x) { return (x + tsqr::kAlign - 1) / tsqr::kAlign * tsqr::kAlign; }

static tsqr_opts orth_opts(const tsqr_opts *o) {
    tsqr_opts q;
    if (o) q = *o;
    else tsqr_default_opts(&q);
    q.keep_q = 1;
    q.prec = TSQR_F64;
    return q;
}

TSQR_API size_t tsqr_block_orth_workspace_bytes(int64_t m, int64_t nv, int64_t b, const tsqr_opts *o) {
    if (nv < 0 || b < 1 || b > tsqr::kMaxPanel || nv + b > m) return 0;
    const tsqr_opts q = orth_opts(o);
    const size_t ws = tsqr_workspace_bytes(m, b, &q);
    if (!ws) return 0;
    const size_t part = sizeof(double) * (size_t)tsqr::proj_blocks(m) * (size_t)nv * (size_t)b;
    return orth_align(ws) + orth_align(part) + orth_align(sizeof(double) * (size_t)nv * (size_t)b);
}

TSQR_API int tsqr_block_orth(int64_t m, int64_t nv, const double *V, int64_t ldv, int64_t b, double *W,
                             int64_t ldw, double *H, int64_t ldh, double *R, int64_t ldr, const tsqr_opts *o,
                             void *dwork, size_t work_bytes, void *stream) {
    if (m < 1) return -1;
    if (nv < 0 || nv + b > m) return -2;
    if (nv > 0 && !V) return -3;
    if (nv > 0 && ldv < m) return -4;
    if (b < 1 || b > tsqr::kMaxPanel) return -5;
    if (!W) return -6;
    if (ldw < m) return -7;
    if (nv > 0 && !H) return -8;
    if (nv > 0 && ldh < nv) return -9;
    if (!R) return -10;
    if (ldr < b) return -11;
    const tsqr_opts q = orth_opts(o);
    Plan plan;
    int rc = tsqr::make_plan(m, b, &q, &plan);
    if (rc) return -12;
    const size_t need = tsqr_block_orth_workspace_bytes(m, nv, b, &q);
    if (!dwork || need == 0 || work_bytes < need || (reinterpret_cast<uintptr_t>(dwork) % tsqr::kAlign))
        return TSQR_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(dwork);
    const size_t ws = orth_align(plan.total);
    double *Hpart = reinterpret_cast<double *>(base + ws);
    double *H2 = reinterpret_cast<double *>(
        base + ws + orth_align(sizeof(double) * (size_t)tsqr::proj_blocks(m) * (size_t)nv * (size_t)b));
    if (nv > 0) {
        const int iv = (int)nv, ib = (int)b;
        // two passes of block classical Gram-Schmidt
        TRY(tsqr::launch_proj(V, ldv, iv, W, ldw, ib, m, Hpart, H, ldh, nullptr, 0, st));
        TRY(tsqr::launch_proj_update(V, ldv, iv, H, ldh, W, ldw, ib, m, st));
        TRY(tsqr::launch_proj(V, ldv, iv, W, ldw, ib, m, Hpart, H2, nv, H, ldh, st));
        TRY(tsqr::launch_proj_update(V, ldv, iv, H2, nv, W, ldw, ib, m, st));
    }
    // TSQR of the projected block; its thin Q replaces it
    tsqr_factors_s f;
    rc = tsqr::factor_into(&f, m, b, W, ldw, &q, dwork, ws, st);
    if (rc) return rc;
    rc = tsqr_form_q(&f, W, ldw, stream);
    if (!rc) rc = tsqr_get_r(&f, R, ldr, stream);
    return rc;
}

TSQR_API int tsqr_last_refine_iters(tsqr_factors f, void *stream) {
    (void)stream;
    return f ? f->last_refine : -1;
}

TSQR_API int64_t tsqr_tree_schedule(int64_t P, int tree, int64_t *left, int64_t *right, int64_t cap) {
    if (P < 1) return -1;
    if (tree != TSQR_TREE_FLAT && tree != TSQR_TREE_BINARY && tree != TSQR_TREE_QUAD && tree != TSQR_TREE_XCD)
        return -2;
    auto s = tsqr::tree_schedule(P, tree);
    for (int64_t i = 0; i < (int64_t)s.size() && i < cap; ++i) {
        if (left) left[i] = s[i].first;
        if (right) right[i] = s[i].second;
    }
    return (int64_t)s.size();
}

TSQR_API int tsqr_free(tsqr_factors f) {
    delete f;
    return 0;
}

TSQR_API const char *tsqr_strerror(int code) {
    if (code == 0) return "success";
    if (code == TSQR_ERR_WORKSPACE) return "workspace missing, misaligned or too small";
    if (code == TSQR_ERR_STATE) return "factor handle cannot serve this call (keep_q = 0?)";
    if (code == TSQR_ERR_UNSUPPORTED) return "shape outside the supported scope (n <= 1024; mixed precision and the condition estimate n <= 256)";
    if (code <= -1000) return "HIP runtime error (code = -1000 - hipError_t)";
    if (code < 0) return "invalid argument (code = -index of the argument)";
    return "unknown";
}

}  // extern "C"
