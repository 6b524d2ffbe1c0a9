// kernels.h -- launch interface of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace tsqr {

// Geometry of one panel TSQR as the kernels see it.
struct PanelArgs {
    int64_t m;      // rows of the panel
    int64_t mb;     // rows per domain
    int64_t P;      // domains
    int64_t cpd;    // chunks per full domain
    int64_t chunk;  // rows per chunk
    int64_t extra;  // load-balanced partition: domains 0 .. extra-1 hold one
                    // chunk more than mb (then mb = cpd chunks); 0 otherwise
    const int64_t *wtab;  // weighted partition: first chunk of every domain
                          // (P + 1 entries, device), else nullptr
    int64_t maxch;  // most chunks of any domain
    int n;          // columns (<= 64)
    int ns;         // column slots per thread of the leaf kernel
};

// Domain d holds rows [dom_row0(d), dom_row0(d) + dom_rows(d)) of the panel,
// and its chunks' T factors sit in slots dom_chunk0(d), ... of the panel's
// chunk array.  The last domain ends at row m (it may be shorter than mb, or
// longer when a short remainder was merged into it).
// (Device code only for a weighted partition, whose table is in device
// memory.)
__host__ __device__ inline int64_t dom_row0(const PanelArgs &pa, int64_t d) {
    if (pa.wtab) return pa.wtab[d] * pa.chunk;
    return d * pa.mb + (d < pa.extra ? d : pa.extra) * pa.chunk;
}
__host__ __device__ inline int64_t dom_rows(const PanelArgs &pa, int64_t d) {
    if (d == pa.P - 1) return pa.m - dom_row0(pa, d);
    if (pa.wtab) return (pa.wtab[d + 1] - pa.wtab[d]) * pa.chunk;
    return pa.mb + (d < pa.extra ? pa.chunk : 0);
}
__host__ __device__ inline int64_t dom_chunk0(const PanelArgs &pa, int64_t d) {
    if (pa.wtab) return pa.wtab[d];
    return d * pa.cpd + (d < pa.extra ? d : pa.extra);
}

// The domain holding chunk slot g of the panel and the chunk's index in it.
__host__ __device__ inline void dom_of_chunk(const PanelArgs &pa, int64_t g, int64_t &dom, int64_t &ch) {
    if (pa.wtab) {
        int64_t lo = 0, hi = pa.P - 1;   // the last d with wtab[d] <= g
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (pa.wtab[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        dom = lo;
    } else {
        const int64_t big = pa.extra * (pa.cpd + 1);   // slots of the longer domains
        dom = g < big ? g / (pa.cpd + 1) : pa.extra + (g - big) / pa.cpd;
        if (dom > pa.P - 1) dom = pa.P - 1;            // a merged last domain
    }
    ch = g - dom_chunk0(pa, dom);
}

// Most chunks any domain has (from the plan).
inline int64_t max_domain_chunks(const PanelArgs &pa) { return pa.maxch; }

// One tree level: chain c = 0..chains-1 starts at
//     left = (c / width) * span + c % width
// and takes rights left + q * stride for q = 1.. while q * stride < span and
// the right is < P (width = 1: left = c * span; the XCD-local levels of the
// hierarchical tree have width = the XCD count, so that consecutive chains
// -- dispatched round-robin over the XCDs -- reduce the domains of their own
// XCD).  A chain whose left is >= P does nothing.
struct TreeArgs {
    int64_t stride;
    int64_t span;
    int64_t chains;
    int64_t width = 1;
};

__host__ __device__ inline int64_t tree_left(const TreeArgs &ta, int64_t c) {
    return (c / ta.width) * ta.span + c % ta.width;
}

// All levels of a reduction tree (bottom first), passed by value.
constexpr int kMaxTreeLevels = 64;
struct TreePath {
    int nlev;
    int64_t stride[kMaxTreeLevels];
    int64_t span[kMaxTreeLevels];
};

size_t factor_smem_bytes();

// ---------------------------------------------------------------------------
// Batched path: one descriptor per matrix (single panel, n <= 64, one
// right-hand side), resident in device memory.  Batched kernels take a list
// of matrix indices and run grid.y = list length, grid.x = the largest count
// of work items (domains, chains, row blocks) of any listed matrix; a
// workgroup whose item does not exist for its matrix returns at once.
constexpr int kMaxLevels = 32;

struct BMat {
    // caller's memory
    const double *A;
    int64_t lda;
    const double *b;      // one right-hand side (m)
    double *R;            // n x n output, leading dimension n
    double *x;            // n output
    double *resid;        // one double
    int32_t *info;        // one int32
    // workspace
    double *V;            // m x n reflectors (FP64 matrices)
    float *V32;           // m x n reflectors (mixed matrices)
    double *Tc, *Rdom, *Tnode, *dsign;
    double *F;            // m: Q^T f / correction vector
    double *Rr;           // m: refined residual (mixed)
    double *Xw;           // n: running solution
    double *gpart;        // nb x n partial A^T r
    double *rpart;        // nb x 2 partial ||b - A x||^2 and ||b - r - A x||^2
    double *hist;         // [0] last relative correction, [1] residual norm (FP64), [2] ||A^T r|| (mixed)
    int32_t *status;      // [0] sweeps done, [1] converged
    PanelArgs pa;
    double *Pc, *Zc;      // per chunk n x 1 blocks of the few-column apply
    int64_t tchunks;      // chunks over all domains
    int prec;             // 0 FP64, 1 mixed
    int nlev;             // tree levels
    int nb;               // row blocks of the residual pass
    int pad;
    TreeArgs lev[kMaxLevels];
};

// factor.hip
// keep_q of the leaf launches: 0 no Q, 1 each chunk's T built in the leaf,
// 2 each chunk's Gram entries and tau stored instead, for launch_chunk_t.
// T of every chunk from what a keep_q == 2 leaf stored.
hipError_t launch_chunk_t(double *Tc, const PanelArgs &pa, int64_t total_chunks, hipStream_t st);
hipError_t launch_leaf(const double *A, int64_t lda, double *V, int64_t ldv, double *Tc, double *Rdom,
                       const PanelArgs &pa, int keep_q, hipStream_t st);
hipError_t launch_tree_level(double *Rdom, double *Tnode, const PanelArgs &pa, const TreeArgs &ta,
                             int keep_q, hipStream_t st);
// T of every tree node (nodes 1 .. P - 1) from the Gram entries and tau the
// levels stored; launched once after the last level when Q is kept.
hipError_t launch_tree_t(double *Tnode, const PanelArgs &pa, hipStream_t st);
// The same leaf with the reflectors stored in FP32 (mixed precision).
hipError_t launch_leaf32(const double *A, int64_t lda, float *V, int64_t ldv, double *Tc, double *Rdom,
                         const PanelArgs &pa, int keep_q, hipStream_t st);
hipError_t launch_sign_normalise(const double *Rroot, int n, double *Rout, int64_t ldr, int row_off,
                                 int col_off, double *dsign, hipStream_t st);

// apply.hip: Q^T (trans = 1) or Q (trans = 0) of a panel's leaves / tree on
// k columns.  Bsrc may differ from B (out of place) or equal it.
hipError_t launch_leaf_apply(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                             const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                             int trans, hipStream_t st);
// apply_mfma.hip: the same leaf application on FP64 matrix cores
// (16 columns of B per workgroup).
hipError_t launch_leaf_apply_m(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                               const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                               int trans, hipStream_t st);
// The same with FP32 reflectors on FP32 matrix cores (mixed precision).
hipError_t launch_leaf_apply_m32(const float *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                                 const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                                 int trans, hipStream_t st);
// Three-pass leaf apply for k <= 16 columns, in place on B (pass 1 P_c =
// V_c^T B_c for every chunk, pass 2 the per-domain chain on n x k blocks,
// pass 3 B_c -= V_c Z_c for every chunk).  Pc and Zc hold one n x k block
// per chunk.
constexpr int kApply3MaxCols = 16;
hipError_t launch_leaf_apply3(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa, double *B,
                              int64_t ldb, int64_t k, int trans, double *Pc, double *Zc, hipStream_t st);
hipError_t launch_leaf_apply3_32(const float *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                                 double *B, int64_t ldb, int64_t k, int trans, double *Pc, double *Zc,
                                 hipStream_t st);
hipError_t launch_tree_apply(const double *Rdom, const double *Tnode, const PanelArgs &pa,
                             const TreeArgs &ta, double *B, int64_t ldb, int64_t k, int trans,
                             hipStream_t st);
// Scale rows [0, n) of B (k columns) by the signs d.
hipError_t launch_scale_rows(double *B, int64_t ldb, int n, int64_t k, const double *d, hipStream_t st);

// formq.hip: thin Q of a single-panel factorization (n <= 64).
hipError_t launch_seed_root(double *S, int n, const double *dsign, hipStream_t st);
hipError_t launch_tree_down_top(const double *Rdom, const double *Tnode, const double *dsign, double *S,
                                const PanelArgs &pa, const TreePath &tp, int lstop, int64_t dstride,
                                hipStream_t st);
hipError_t launch_tree_down(const double *Rdom, const double *Tnode, double *S, const PanelArgs &pa,
                            const TreeArgs &ta, hipStream_t st);
hipError_t launch_form_leaf(const double *V, int64_t ldv, const double *Tc, const double *S,
                            const PanelArgs &pa, double *Q, int64_t ldq, hipStream_t st);

// misc.hip
hipError_t launch_fill_identity_signs(double *Q, int64_t ldq, int64_t m, int n, const double *d,
                                      hipStream_t st);
// p[0..count) = value (a kernel, so it is safe inside captured graphs).
hipError_t launch_fill(double *p, int64_t count, double value, hipStream_t st);
hipError_t launch_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                       int64_t cols, hipStream_t st);
// TSLU (tslu.hip): candidate rows per domain into cand (P x b, int32), the
// tree levels, then ipiv, U (b x b), L (m x b) and dinfo; L11 is a 64 x 64
// scratch block.
hipError_t launch_tslu(const double *A, int64_t lda, const PanelArgs &pa, const std::vector<TreeArgs> &levels,
                       int b, int32_t *cand, double *L11, double *L, int64_t ldl, double *U, int64_t ldu,
                       int64_t *ipiv, int32_t *dinfo, hipStream_t st);

// CALU pieces: clear the info word; after a panel's TSLU (pivot rows piv,
// L (mr x b, ld ldl), U (b x b, ld ldu), its info word pinfo): the row
// interchanges (meta: kCaluMetaWords int32 of device scratch;
// ipiv_out[k..k+b-1]), their application outside the panel, the packed
// panel, U12 and the trailing update.
constexpr int kCaluMetaWords = 324;
hipError_t launch_calu_clear(int32_t *dinfo, hipStream_t st);
hipError_t launch_calu_panel_rest(double *A, int64_t lda, int64_t m, int64_t n, int64_t k, int b,
                                  const int64_t *piv, int32_t *meta, int64_t *ipiv_out, const int32_t *pinfo,
                                  int32_t *dinfo, const double *L, int64_t ldl, const double *U, int64_t ldu,
                                  hipStream_t st);

// In-place Cholesky A = L L^T of the lower triangle of an n x n SPD matrix
// (lda >= n); *dinfo (device) <- 0 or the order of the first leading minor
// that is not positive definite.
hipError_t launch_cholesky(int64_t n, double *A, int64_t lda, int32_t *dinfo, hipStream_t st);

// kappa_1(R) estimate of an n x n upper-triangular R (ld n, n <= 256) into
// *kappa (device): one wave.
hipError_t launch_cond_est(const double *R, int n, double *kappa, hipStream_t st);
hipError_t launch_lsq_finish(const double *R, int n, const double *C, int64_t ldc, int64_t m, int64_t k,
                             double *X, int64_t ldx, double *resid, int32_t *dinfo, double *partial,
                             hipStream_t st);

// orth.hip: block Gram-Schmidt projections against an orthonormal basis.
constexpr int kProjMaxBlocks = 512;   // row blocks of the partial products
int proj_blocks(int64_t m);
// H = V^T W (nv x b, ld ldh) through per-block partials (Hpart: proj_blocks(m)
// x nv x b doubles); if Hacc, also Hacc += H.
hipError_t launch_proj(const double *V, int64_t ldv, int nv, const double *W, int64_t ldw, int b, int64_t m,
                       double *Hpart, double *H, int64_t ldh, double *Hacc, int64_t ldacc, hipStream_t st);
// W -= V H.
hipError_t launch_proj_update(const double *V, int64_t ldv, int nv, const double *H, int64_t ldh, double *W,
                              int64_t ldw, int b, int64_t m, hipStream_t st);

// refine.hip: FP64 pieces of the mixed-precision least-squares refinement.
int resid_blocks(int64_t m);
hipError_t launch_lsq_resid(const double *A, int64_t lda, int64_t m, int n, const double *B, int64_t ldb,
                            const double *X, int64_t ldx, const double *Rr, double *F, int k,
                            double *gpart, double *rpart, int nblocks, hipStream_t st);
hipError_t launch_lsq_refine(const double *R, int n, double *F, int64_t m, int k, const double *gpart,
                             int nblocks, double *X, int64_t ldx, double tol, int32_t *status,
                             double *hist, double *gnorm, hipStream_t st);
hipError_t launch_axpy(double *y, const double *x, int64_t count, hipStream_t st);
hipError_t launch_status_init(int32_t *status, double *hist, int k, hipStream_t st);
hipError_t launch_mixed_final(const double *R, int n, int k, const double *Xw, double *X, int64_t ldx,
                              double *resid, int32_t *dinfo, int merge, const double *rpart, int nblocks,
                              const double *gnorm, double *eta_out, hipStream_t st);

// batched launches (device descriptor array `mats`, index list `list` of
// `cnt` entries, `gx` = grid.x as described above)
hipError_t launch_leaf_b(const BMat *mats, const int *list, int cnt, int64_t gx, int ns, hipStream_t st);
hipError_t launch_tree_b(const BMat *mats, const int *list, int cnt, int64_t gx, int ns, int level,
                         hipStream_t st);
hipError_t launch_tree_t_b(const BMat *mats, const int *list, int cnt, int64_t maxP, hipStream_t st);
hipError_t launch_sign_b(const BMat *mats, const int *list, int cnt, hipStream_t st);
// Q^T (trans = 1) or Q (trans = 0) on F, leaves, in three chunk-parallel
// passes (grid.x: max_chunks for passes 1 and 3, max_p for pass 2); sweep > 0
// skips converged matrices.
hipError_t launch_apply3_b(const BMat *mats, const int *list, int cnt, int64_t max_chunks, int64_t max_p,
                           int trans, int sweep, hipStream_t st);
// one tree level; step counts from the bottom (trans = 1) or the top (0)
hipError_t launch_tree_apply_b(const BMat *mats, const int *list, int cnt, int64_t gx, int trans, int step,
                               int sweep, hipStream_t st);
hipError_t launch_scale_b(const BMat *mats, const int *list, int cnt, int sweep, hipStream_t st);
hipError_t launch_lsq_init_b(const BMat *mats, const int *list, int cnt, int64_t gx, hipStream_t st);
hipError_t launch_resid_b(const BMat *mats, const int *list, int cnt, int64_t gx, int sweep, hipStream_t st);
hipError_t launch_refine_b(const BMat *mats, const int *list, int cnt, int sweep, double tol, hipStream_t st);
hipError_t launch_axpy_b(const BMat *mats, const int *list, int cnt, int64_t gx, int sweep, hipStream_t st);
hipError_t launch_final_b(const BMat *mats, const int *list, int cnt, hipStream_t st);

}  // namespace tsqr
