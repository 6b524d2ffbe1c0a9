/*
 * tsqr.h -- C ABI of the MI355X (gfx950) TSQR library.
 *
 * The library factors a tall-and-skinny m x n FP64 matrix (m >= n) with TSQR,
 * the panel factorization of Communication-Avoiding QR described in Sec. 2.3
 * of Agullo, Coti, Dongarra, Herault and Langou, "QR Factorization of Tall and
 * Skinny Matrices in a Grid Computing Environment" (arXiv 0912.2572):
 *   1. the rows are split into P contiguous domains (block rows);
 *   2. every domain gets a Householder QR (Sec. 2.2: H = I - tau v v^T,
 *      blocked as H_1...H_b = I - V T V^T with T upper triangular);
 *   3. the P triangular factors are reduced pairwise, R = qr([R_1; R_2]).R,
 *      up a binary, 4-ary or flat tree (Sec. 2.3);
 *   4. R is made unique by a nonnegative diagonal (Sec. 2.2: QR is unique
 *      once diag(R) > 0), i.e. R <- D R and Q <- Q D, D = diag(sgn R_jj),
 *      sgn(0) = +1.
 * The same tree applies Q^T, applies Q, forms the thin Q, and solves least
 * squares min ||A x - b||_2 (the paper notes QR as the first step toward
 * least squares; the solve is the textbook x = R^{-1} Q_1^T b).
 *
 * Conventions for every entry point:
 *   - matrices are column-major FP64 in DEVICE memory unless stated;
 *   - the caller owns all device memory (A, B, X, Q, R and the workspace);
 *     the library never allocates device memory in these calls except the
 *     serving front-end, which documents its own allocations;
 *   - calls are asynchronous and ordered on the given HIP stream, passed as
 *     an opaque pointer (hipStream_t; NULL = the default stream);
 *   - return value 0 = success; -i = argument i is invalid (1-based, LAPACK
 *     style); TSQR_ERR_WORKSPACE when the workspace is too small;
 *     -1000 - e for a HIP runtime error e.
 *
 * Scope limits: 1 <= n <= 1024 (TSQR_MIXED and tsqr_cond_estimate:
 * n <= 256), n <= m <= 2^31 - 1, domain rows >= n.  Wider than 64 columns,
 * the matrix is factored in 64-column panels (Sec. 2.3's CAQR structure:
 * each panel a TSQR of the rows below the previous ones, its Q^T applied to
 * the columns to its right), so square matrices up to 1024 are covered.
 */
#ifndef TSQR_H_
#define TSQR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSQR_API __attribute__((visibility("default")))

/* Reduction-tree shapes (Sec. 2.3: binary and flat trees; the k-ary tree
   generalises the binary one).  TSQR_TREE_XCD is the hierarchical tree of
   Sec. 2.3 (Fig. 2) and Sec. 3 with an XCD of the GPU as a cluster: domain d
   belongs to XCD d mod 8 (the leaves are dispatched round-robin over the 8
   XCDs); a binary tree reduces each XCD's domains first, so those
   triangles stay in that XCD's L2, and a binary tree then reduces the 8 XCD
   roots: 7 combines cross an XCD boundary (G - 1 for G groups).  Results
   always land in the lower-index child, so the root is domain 0 and its
   first n rows hold the top of Q^T B. */
enum { TSQR_TREE_FLAT = 0, TSQR_TREE_BINARY = 2, TSQR_TREE_QUAD = 4, TSQR_TREE_XCD = 8 };

/* Arithmetic of the factorization.  TSQR_F64: everything in FP64.
   TSQR_MIXED: reflector generation (norms, beta, tau), the leaf and tree
   Householder steps and every residual in FP64; the reflectors are stored in
   FP32 and every application of Q or Q^T (the trailing updates between
   64-column panels, apply_qt/apply_q/form_q, the solves inside least
   squares) runs on FP32 matrix cores with FP32 accumulation.  The factor is
   then FP32-accurate (R exact to FP64 rounding for n <= 64, where no FP32
   trailing update runs; Q orthogonal to about 1e-6), and tsqr_lsq_solve is
   brought back to FP64 accuracy by iterative refinement of the augmented
   system [I A; A^T 0][r; x] = [b; 0] with FP64 residuals (Bjorck). */
enum { TSQR_F64 = 0, TSQR_MIXED = 1 };

/* Error codes beyond the LAPACK-style -i. */
enum {
    TSQR_ERR_WORKSPACE = -900,   /* workspace pointer NULL or too small      */
    TSQR_ERR_STATE = -901,       /* handle not usable for this call (e.g. a */
                                 /* factor made with keep_q = 0)             */
    TSQR_ERR_UNSUPPORTED = -902  /* shape outside the documented scope       */
};

typedef struct {
    int64_t row_block;       /* mb, rows per domain; 0 = library default.   */
                             /* Must be >= n.  P = ceil(m / mb); a last     */
                             /* domain shorter than n rows is merged into   */
                             /* the one before it.                          */
    int32_t tree;            /* TSQR_TREE_*                                  */
    int32_t prec;            /* TSQR_F64 or TSQR_MIXED                       */
    int32_t keep_q;          /* 1: store the reflectors (needed by apply/   */
                             /* form_q/lsq); 0: R only, the paper's         */
                             /* measured mode (Sec. 1).                     */
    int32_t lsq_max_rhs;     /* largest k passed to tsqr_lsq_solve (>= 1)   */
    int32_t refine_max_iter; /* mixed: refinement sweeps after the first   */
                             /* solve (cap)                                */
    int32_t domains;         /* 0: the row_block partition above.  > 0:     */
                             /* load-balanced partition (Sec. 3: rows per  */
                             /* domain follow the processing power behind  */
                             /* it; the compute units of one GPU are equal,*/
                             /* so the shares are equal): this many        */
                             /* domains of whole leaf chunks (chunk_rows   */
                             /* of tsqr_plan_info), the first C mod P of   */
                             /* them one chunk longer (C = ceil(m / chunk) */
                             /* chunks), the last ending at row m.  Fewer  */
                             /* domains are used when C < P or when the    */
                             /* last would be shorter than n rows.  -1:    */
                             /* one domain per leaf workgroup the GPU      */
                             /* holds at once (256 compute units times the */
                             /* leaf workgroups per unit for this n).      */
                             /* Needs row_block = 0.  Each 64-column panel */
                             /* of a wider matrix is balanced on its own.  */
    double refine_tol;       /* stop when the error left, estimated as
                                ||dx|| times the sweep-to-sweep contraction
                                ||dx|| / ||dx_prev||, is <= tol ||x||       */
    double route_kappa;      /* mixed: the first tsqr_lsq_solve of a factor
                                estimates kappa_1(R) (tsqr_cond_estimate);
                                above route_kappa (or not finite) it factors
                                A again in FP64 in the same workspace, and
                                that solve and every later call on the
                                handle use the FP64 factor, so an
                                ill-conditioned problem skips a long
                                refinement.  0 = never (default); >= 0.    */
    const int64_t *domain_weights; /* NULL (default), or num_weights      */
    int64_t num_weights;     /* integer powers 1 .. 2^31 (host memory,    */
                             /* read while planning; at most 2^31 of them)*/
                             /* while planning): that many domains, the   */
                             /* rows apportioned to the powers in whole   */
                             /* leaf chunks (C = ceil(m / chunk) chunks;  */
                             /* floor(C w_d / W) each, the rest one each  */
                             /* to the largest remainders C w_d mod W,    */
                             /* ties to the lower index), the last domain */
                             /* ending at row m: Sec. 3's rows in         */
                             /* proportion to each domain's processing    */
                             /* power, e.g. the share of its XCD (domain  */
                             /* d runs on XCD d mod 8) other work leaves. */
                             /* Every domain must get a chunk and at least*/
                             /* n rows, else -5.  Needs row_block = 0 and */
                             /* domains = 0.  The factorization copies    */
                             /* the domain table (8 (P + 1) bytes) from   */
                             /* host memory on its stream, so it cannot   */
                             /* be captured in a HIP graph; not accepted  */
                             /* by tsqr_factor_solve_noalloc.             */
} tsqr_opts;

/* Opaque host handle describing one factorization.  It points into the
   caller's workspace, which must outlive it and must not be reused by
   another factorization while the handle is in use. */
typedef struct tsqr_factors_s *tsqr_factors;

/* Fill *o with the defaults: row_block 0 (library default), binary tree,
   FP64, keep_q 1, lsq_max_rhs 8, refine_max_iter 30, domains 0,
   refine_tol 1e-14, route_kappa 0, no domain weights. */
TSQR_API void tsqr_default_opts(tsqr_opts *o);

/* Bytes of device workspace tsqr_factor needs for an m x n problem with
   options o (NULL = defaults).  Returns 0 for invalid arguments. */
TSQR_API size_t tsqr_workspace_bytes(int64_t m, int64_t n, const tsqr_opts *o);

/* Factor A (m x n, leading dimension lda >= m, device, not modified):
   partition (step 1), leaf QR of every domain (step 2), tree (step 3) and
   sign normalisation (step 4), all on `stream`.  dwork: device workspace of
   at least tsqr_workspace_bytes() bytes, 256-byte aligned.  *out receives a
   new host handle (free it with tsqr_free).
   Errors: -1 m, -2 n, -3 A NULL, -4 lda, -5 opts (row_block < n, bad tree or
   precision, domains < -1 or set together with row_block),
   TSQR_ERR_WORKSPACE, -1000-e on a HIP error. */
TSQR_API int tsqr_factor(int64_t m, int64_t n, const double *A, int64_t lda,
                         const tsqr_opts *o, void *dwork, size_t work_bytes,
                         void *stream, tsqr_factors *out);

/* Copy the sign-normalised R (n x n upper triangular, zeros below the
   diagonal, diag >= 0) to R (device, leading dimension ldr >= n).
   Defined by Sec. 2.2 (A = QR with R upper triangular; unique once the
   diagonal is made positive).  Errors: -1 handle, -2 R NULL, -3 ldr. */
TSQR_API int tsqr_get_r(tsqr_factors f, double *R, int64_t ldr, void *stream);

/* B <- Q^T B for the factor's full m x m orthogonal Q (k columns, device,
   ldb >= m).  Rows 0..n-1 of the result equal Q_1^T B for the
   sign-normalised thin Q_1, whatever the tree or partition; rows n..m-1 are
   a valid complement for this factor's Q and depend on its representation.
   Defined by Sec. 2.3 (Q is kept implicitly as the leaves' and the tree
   nodes' reflectors; Q^T is applied leaves first, then up the tree in the
   factorization's order) and Sec. 4, Property 1 (the Q work has the
   structure of the R work).  Errors: -1 handle, TSQR_ERR_STATE (keep_q = 0),
   -2 k < 0, -3 B NULL, -4 ldb. */
TSQR_API int tsqr_apply_qt(tsqr_factors f, int64_t k, double *B, int64_t ldb, void *stream);

/* B <- Q B, the inverse of tsqr_apply_qt (same representation): the tree
   top-down, then the leaves (Sec. 2.3).  Errors as tsqr_apply_qt. */
TSQR_API int tsqr_apply_q(tsqr_factors f, int64_t k, double *B, int64_t ldb, void *stream);

/* Thin Q (m x n, device, ldq >= m), sign-normalised so that A = Q R with
   diag(R) >= 0 and Q^T Q = I.  Defined by Sec. 1 (Q formed explicitly, at
   twice the cost of R: Table 2) and Sec. 2.3 (Q = [I_n; 0] pushed down the
   tree, then through each leaf).  Errors: -1 handle, TSQR_ERR_STATE, -2 Q
   NULL, -3 ldq.
   Concurrency: calls on one factor are ordered by the caller (one stream,
   or events).  One exception: for an FP64 factor with n <= 64 this call only
   reads the factor and writes Q and its own workspace blocks (the top-down
   tree blocks), so once tsqr_factor has completed it may run on another
   stream at the same time as tsqr_lsq_solve, tsqr_apply_qt or tsqr_apply_q
   on the same factor. */
TSQR_API int tsqr_form_q(tsqr_factors f, double *Q, int64_t ldq, void *stream);

/* Least squares min ||A x_j - b_j||_2 for k <= opts.lsq_max_rhs right-hand
   sides: X = R^{-1} (Q^T B)[0:n], resid[j] = ||(Q^T B)[n:m, j]||_2.  The
   paper names QR as the first step toward least squares (Sec. 1); the solve
   is the textbook one through the factors of Sec. 2.3.
   A (m x n, lda) is the matrix that was factored; it is read only by the
   mixed-precision refinement (required there: -2 when NULL), which
   synchronises `stream` once per sweep to read its convergence flag and
   reports resid[j] = ||b_j - A x_j||_2 computed in FP64 from the last
   sweep's residual pass.  B (m x k, ldb) is not modified.  X (n x k,
   ldx >= n) and resid (k doubles, may be NULL) are device outputs.
   dinfo (device int32, may be NULL) receives 0, or j+1 when R_jj == 0
   exactly (X is then left untouched, LAPACK dtrtrs convention), or -2 when
   a residual is not finite, or (mixed precision only) -3 when the
   refinement ended -- stalled, or after refine_max_iter sweeps -- with an
   upper bound on the backward error eta = ||A^T (b - A x)|| /
   (||A||_F (||A||_F ||x|| + ||b - A x||)) above 1e-12 for some right-hand
   side: X is then written but is not FP64-accurate (the bound of every
   right-hand side is available from tsqr_lsq_backward_error).  dinfo is
   valid after the stream synchronises.
   Errors: -1 handle, TSQR_ERR_STATE, -2 A (mixed: NULL), -3 lda, -4 k,
   -5 B NULL, -6 ldb, -7 X NULL, -8 ldx. */
TSQR_API int tsqr_lsq_solve(tsqr_factors f, const double *A, int64_t lda, int64_t k,
                            const double *B, int64_t ldb, double *X, int64_t ldx,
                            double *resid, int32_t *dinfo, void *stream);

/* tsqr_factor, tsqr_lsq_solve and (Q != NULL) tsqr_form_q in one call, with
   the arguments and results of those three (*out: the factor handle, as
   from tsqr_factor; opts.keep_q must be set: TSQR_ERR_STATE otherwise).
   Least squares through TSQR applies Q^T to B leaf by leaf and then up the
   tree, the same traversal as the factorization (Sec. 2.3): the leaf pass of
   Q^T B needs only the leaf factors, so for an FP64 factor of one panel
   (n <= 64) it runs on a second stream, owned by the library, while the
   tree is factored, and the solve's tree pass then runs beside the thin Q.
   `stream` waits for that stream before the call's work ends, so the call is
   ordered on `stream` like any other.  The second stream and its events are
   created on the current device at the first call and kept until the
   process ends; concurrent calls from several host threads are serialised
   while they enqueue.  Other factors run the three calls in order on
   `stream`.  Results are bitwise those of the three separate calls.
   Errors: those of tsqr_factor (-1 .. -5, TSQR_ERR_WORKSPACE), then -8 k,
   -9 B NULL, -10 ldb, -11 X NULL, -12 ldx, -16 ldq, -18 out NULL, and the
   errors of the solve and the thin Q. */
TSQR_API int tsqr_factor_solve(int64_t m, int64_t n, const double *A, int64_t lda,
                               const tsqr_opts *o, void *dwork, size_t work_bytes,
                               int64_t k, const double *B, int64_t ldb, double *X, int64_t ldx,
                               double *resid, int32_t *dinfo, double *Q, int64_t ldq,
                               void *stream, tsqr_factors *out);

/* Bytes of the device scratch array behind tsqr_factor_solve_noalloc (one
   per GPU, held from the library's load until the process ends). */
#define TSQR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
   factorization, least squares and, when Q / R are not NULL, the thin Q and
   R of one matrix, with no allocation and no handle.  The arguments and
   results are those of tsqr_factor_solve followed by tsqr_get_r (R: n x n,
   ldr >= n); the three calls run in order on `stream`, so the results are
   bitwise those of tsqr_factor_solve with the same options.  The workspace
   is the library's own static device array of TSQR_NOALLOC_SCRATCH_BYTES on
   the current GPU (its address is looked up at the first call on each
   device): problems whose tsqr_workspace_bytes(m, n, o) exceeds that size
   return TSQR_ERR_WORKSPACE.  Every call on one GPU shares that array, so
   calls that overlap on one GPU race: order them (one stream, or events).
   Errors: -1 m, -2 n, -3 A NULL, -4 lda, -5 opts, TSQR_ERR_UNSUPPORTED for
   a precision other than TSQR_F64 or for domain weights (their table would
   be copied from host memory), TSQR_ERR_STATE for keep_q = 0,
   TSQR_ERR_WORKSPACE (too large), -6 k, -7 B NULL, -8 ldb, -9 X NULL,
   -10 ldx, -14 ldq, -16 ldr, -1000-e on a HIP error. */
TSQR_API int tsqr_factor_solve_noalloc(int64_t m, int64_t n, const double *A, int64_t lda,
                                       const tsqr_opts *o, int64_t k, const double *B, int64_t ldb,
                                       double *X, int64_t ldx, double *resid, int32_t *dinfo,
                                       double *Q, int64_t ldq, double *R, int64_t ldr, void *stream);

/* Backward-error bounds of the last mixed-precision tsqr_lsq_solve on this
   handle, one per right-hand side (k <= that solve's k), copied to eta
   (device, k doubles) on `stream`: eta_j bounds ||A^T s_j|| / (||A||_F
   (||A||_F ||x_j|| + ||s_j||)) with s_j = b_j - A x_j, from the last
   refinement sweep's FP64 residuals (||A^T s|| <= ||A^T r|| + ||A|| ||b - r
   - A x||, ||A||_F = ||R||_F).  A right-hand side with eta_j > 1e-12 made
   that solve's dinfo -3.  Errors: -1 handle, TSQR_ERR_STATE (FP64 factor,
   or no mixed solve yet), -2 k, -3 eta NULL. */
TSQR_API int tsqr_lsq_backward_error(tsqr_factors f, int64_t k, double *eta, void *stream);

/* ------------------------------------------------------------------------
   Block orthogonalisation: the step block-iterative methods (block Krylov
   solvers, block eigensolvers) repeat to grow an orthonormal basis, with
   TSQR as the stable orthogonalisation of each new block (Scope section and
   Sec. 6 of the paper).  For an orthonormal V (m x nv) and a new block W
   (m x b): two passes of block classical Gram-Schmidt
       H1 = V^T W,  W -= V H1,  H2 = V^T W,  W -= V H2,
   then TSQR of the projected W (opts: row block and tree; FP64, keep_q
   forced) and its sign-normalised thin Q written over W, so that on return
       W_in = V H + Q R  with H = H1 + H2,  [V Q]^T [V Q] = I,  diag(R) >= 0.
   ------------------------------------------------------------------------ */

/* Device workspace for tsqr_block_orth (0 for arguments out of scope:
   b < 1, b > 64, nv < 0, nv + b > m). */
TSQR_API size_t tsqr_block_orth_workspace_bytes(int64_t m, int64_t nv, int64_t b, const tsqr_opts *o);

/* V: m x nv (ldv >= m, orthonormal columns, read only; NULL when nv = 0),
   W: m x b (ldw >= m; in: the new block, out: Q), H: nv x b (ldh >= nv;
   unused when nv = 0), R: b x b (ldr >= b), all device, column-major.
   dwork: >= tsqr_block_orth_workspace_bytes, 256-byte aligned.  Runs on
   `stream`; allocates nothing.  Errors: -1 m, -2 nv (nv < 0 or nv + b > m),
   -3 V NULL, -4 ldv, -5 b (1..64), -6 W NULL, -7 ldw, -8 H NULL, -9 ldh,
   -10 R NULL, -11 ldr, -12 opts, TSQR_ERR_WORKSPACE, -1000-e. */
TSQR_API int tsqr_block_orth(int64_t m, int64_t nv, const double *V, int64_t ldv, int64_t b, double *W,
                             int64_t ldw, double *H, int64_t ldh, double *R, int64_t ldr, const tsqr_opts *o,
                             void *dwork, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
   TSLU: LU of a tall-skinny matrix with tournament pivoting, the extension
   of TSQR's reduction tree to LU that the paper's conclusion names (CALU's
   panel factorization).  The rows are split into domains as for tsqr_factor
   (opts.row_block or opts.domains, opts.tree for the tree); each domain
   picks b candidate pivot rows by Gaussian elimination with partial
   pivoting over stacks of 256 rows (its first 256 rows, then its
   candidates on the next 256 - b rows), and the tree combines candidate
   sets the same way (the left's stacked on the right's).  With ipiv the
   root's rows in pivot order:
     U (b x b, device, ldu >= b): upper triangular, A[ipiv, :] = L11 U
       without further pivoting;
     L (m x b, device, ldl >= m): rows ipiv[k] hold row k of the unit lower
       L11, every other row l_i = a_i U^{-1}; so A = L U with L a row
       permutation of a unit lower trapezoidal matrix;
     ipiv (b, device, int64): the pivot rows of A, in order;
     dinfo (device, one int32, may be NULL): 0, or j + 1 for the first
       U_jj = 0 (that column's l entries are then 0).
   A pivot search takes the largest |entry| of the live rows, ties to the
   earlier stack position; NaNs rank last.  A (m x b, device, lda >= m) is
   not modified.  b <= 64.  Errors: -1 m, -2 b, -3 A NULL, -4 lda, -5 opts,
   -6 L NULL or ldl, -7 U NULL or ldu, -8 ipiv NULL, TSQR_ERR_WORKSPACE,
   TSQR_ERR_UNSUPPORTED for b > 64, -1000-e on a HIP error. */
TSQR_API size_t tsqr_tslu_workspace_bytes(int64_t m, int64_t b, const tsqr_opts *o);
TSQR_API int tsqr_tslu(int64_t m, int64_t b, const double *A, int64_t lda, const tsqr_opts *o,
                       void *dwork, size_t work_bytes, double *L, int64_t ldl, double *U, int64_t ldu,
                       int64_t *ipiv, int32_t *dinfo, void *stream);

/* ------------------------------------------------------------------------
   CALU: LU of an m x n matrix (m >= n) with tournament pivoting, the LU
   counterpart of CAQR that the conclusion names with TSLU.  Panels of 64
   columns; each panel's pivot rows come from TSLU (above: the domains of
   opts for the m - k rows below the diagonal, opts.tree, 256-row stacks),
   become LAPACK-style row interchanges applied to the whole rows, and are
   followed by U12 = L11^{-1} A12 and the trailing update A22 -= L21 U12 on
   the FP64 matrix cores.
   A (m x n, device, column-major, lda >= m): in, the matrix; out, dgetrf's
     packed factors: U on and above the diagonal, the unit lower L strictly
     below, so that P A = L U with P the interchanges;
   ipiv (n, device, int64): row i was interchanged with row ipiv[i]
     (0-based, ipiv[i] >= i), in order i = 0, 1, ...;
   dinfo (device, one int32, required): 0, or j + 1 for the first U_jj that
     is exactly zero (that column's l entries are zero; the factorization
     goes on).
   opts: row_block or domains and tree as for tsqr_factor (weighted domains
   are TSQR_ERR_UNSUPPORTED).  dwork: >= tsqr_calu_workspace_bytes (0 for
   invalid arguments), 256-byte aligned.  Runs on `stream`; allocates
   nothing.  Errors: -1 m < n, -2 n < 1, -3 A NULL, -4 lda, -5 opts, -8
   ipiv NULL, -9 dinfo NULL, TSQR_ERR_WORKSPACE, TSQR_ERR_UNSUPPORTED for
   m >= 2^31 or weighted domains, -1000-e on a HIP error. */
TSQR_API size_t tsqr_calu_workspace_bytes(int64_t m, int64_t n, const tsqr_opts *o);
TSQR_API int tsqr_calu(int64_t m, int64_t n, double *A, int64_t lda, const tsqr_opts *o, void *dwork,
                       size_t work_bytes, int64_t *ipiv, int32_t *dinfo, void *stream);

/* ------------------------------------------------------------------------
   Cholesky factorization A = L L^T of a symmetric positive definite n x n
   matrix: the third one-sided factorization, beside QR and LU, that the
   paper's introduction and conclusion carry the approach over to.
   Blocked right-looking, communication-avoiding in the sequential sense of
   the Cholesky work the conclusion cites: block columns of 256 columns,
   whose trailing update A22 -= L21 L21^T runs on the FP64 matrix cores (the
   trailing matrix is read and written once per block column), each factored
   in 64-column panels (the 64 x 64 diagonal block in one wave, the rows
   below solved against it, 64 rows per workgroup).
   A (n x n, device, column-major, lda >= max(1, n)): in, the lower triangle
   of the SPD matrix (the strict upper triangle is neither read nor
   written); out, L in the lower triangle.
   dinfo (device, one int32, required): 0, or j > 0 when the leading minor
   of order j is not positive definite (its pivot is <= 0 or NaN, LAPACK's
   dpotrf convention).  The columns of L before the 64-column panel that
   holds column j - 1 are then final; the rest of the lower triangle is
   left part-way.
   Runs on `stream`, allocates nothing.  n = 0 only clears dinfo.  Errors:
   -1 n < 0, -2 A NULL, -3 lda, -4 dinfo NULL, TSQR_ERR_UNSUPPORTED for
   n >= 2^31, -1000-e on a HIP error. */
TSQR_API int tsqr_cholesky(int64_t n, double *A, int64_t lda, int32_t *dinfo, void *stream);

/* Estimate of the 1-norm condition number kappa_1(R) = ||R||_1 ||R^{-1}||_1
   of the factor's R (= kappa_1 of A up to the factorization's rounding),
   written to *kappa (device, one double) on `stream`: ||R||_1 times Hager's
   lower bound on ||R^{-1}||_1 with Higham's refinements (at most five pairs
   of triangular solves, then an alternating-sign test vector), so it never
   exceeds kappa_1(R) and is usually within a factor of 3 of it; +inf when R
   has an exactly zero diagonal entry.  One wave of 64 lanes, n <= 256
   (TSQR_ERR_UNSUPPORTED beyond).
   The paper's method is FP64 only; the estimate serves the mixed-precision
   routing (opts.route_kappa).  Errors: -1 handle, -2 kappa NULL. */
TSQR_API int tsqr_cond_estimate(tsqr_factors f, double *kappa, void *stream);

/* Host only: the precision the handle's reflectors are now in (*prec:
   TSQR_F64 after a mixed factor was routed to FP64 by opts.route_kappa) and
   the condition estimate that decided it (*kappa_est, 0 when no routing
   check ran).  Either pointer may be NULL.  Errors: -1 handle. */
TSQR_API int tsqr_route_info(tsqr_factors f, int32_t *prec, double *kappa_est);

/* Number of sweeps (the first solve included) the last mixed-precision
   tsqr_lsq_solve on this handle ran, the largest over its groups of 8
   right-hand sides; 0 for FP64 factors.  Host only; `stream` is unused. */
TSQR_API int tsqr_last_refine_iters(tsqr_factors f, void *stream);

/* Plan introspection (host only, no device work): number of domains
   (Sec. 2.3's partition into P domains), rows per chunk of the leaf kernel
   and number of 64-column panels. */
TSQR_API int tsqr_plan_info(int64_t m, int64_t n, const tsqr_opts *o,
                            int64_t *num_domains, int64_t *chunk_rows, int64_t *num_panels);

/* The domains of the first 64-column panel (Sec. 2.3's partition, or the
   load-balanced one of opts.domains): row0[i] and nrows[i] for i < min(P,
   cap), host only.  Returns P, or the negative argument code of
   tsqr_factor. */
TSQR_API int64_t tsqr_partition(int64_t m, int64_t n, const tsqr_opts *o, int64_t *row0, int64_t *nrows,
                                int64_t cap);

/* The reduction tree as a list of combines (left, right), in execution
   order, for P domains and tree shape `tree` (host only).  Writes at most
   `cap` pairs and returns the number of combines (P - 1), or a negative
   argument code. */
TSQR_API int64_t tsqr_tree_schedule(int64_t P, int tree, int64_t *left, int64_t *right, int64_t cap);

/* Kernel timing with HIP events (for benchmarks).  While enabled, every
   kernel the library enqueues is bracketed by a pair of events recorded on
   the same stream, tagged with the kernel's name.  tsqr_prof_query
   synchronises on the recorded events and returns, for the i-th distinct
   tag (i = 0, 1, ...), its name, launch count and summed milliseconds; it
   returns 0, or -1 once i is past the last tag.  tsqr_prof_enable(0)
   disables and clears.  tsqr_prof_only(tag) restricts the timing to the
   kernels of one tag (a copy of the string is kept; NULL or "" times all),
   so that a timed loop carries two events per launch of that kernel only.
   Process-wide; the calls may come from several host threads (the
   recorded events are kept under a lock). */
TSQR_API int tsqr_prof_enable(int on);
TSQR_API int tsqr_prof_only(const char *tag);
TSQR_API int tsqr_prof_query(int i, const char **name, int64_t *launches, double *ms);

/* ------------------------------------------------------------------------
   Batched TSQR + least squares.  Many independent matrices (n <= 64, one
   right-hand side each, FP64 or mixed per matrix) are factored and solved
   together: every step of the path (leaf QR, each tree level, sign
   normalisation, Q^T b, the solve and the mixed matrices' refinement
   sweeps) is one launch over all matrices at once, and the whole sequence
   is captured once into a HIP graph and replayed.  Row-block size and tree
   arity come from a tuning table (tsqr_autotune) keyed by (n, precision):
   a matrix's plan depends only on its own (m, n, precision), never on the
   rest of the batch.
   ------------------------------------------------------------------------ */

/* One tuning-table entry: applies to matrices of precision `prec` with
   n <= n_max (the entry with the smallest such n_max wins). */
typedef struct {
    int32_t n_max;
    int32_t prec;
    int64_t row_block;   /* rows per domain (raised to n when smaller)     */
    int32_t tree;        /* TSQR_TREE_*                                    */
    int32_t reserved;
} tsqr_tune_entry;

/* One matrix of a batch.  All pointers are device pointers the caller owns;
   A (m x n, lda >= m) and b (m) are read only. */
typedef struct {
    int64_t m, n;        /* 1 <= n <= 64, n <= m <= 2^31 - 1                */
    int32_t prec;        /* TSQR_F64 or TSQR_MIXED                          */
    int32_t reserved;
    const double *A;
    int64_t lda;
    const double *b;
    double *R;           /* n x n output (leading dimension n), diag >= 0   */
    double *x;           /* n output: argmin ||A x - b||_2                  */
    double *resid;       /* 1 output: ||b - A x||_2 (FP64 matrices: the    */
                         /* norm of (Q^T b)[n:m])                           */
    int32_t *info;       /* 1 output: 0, j+1 for R_jj == 0 (x untouched),  */
                         /* -2 for a non-finite residual, -3 (mixed) when   */
                         /* the refined x's backward-error bound is above   */
                         /* 1e-12 (see tsqr_lsq_solve)                      */
} tsqr_batch_item;

typedef struct tsqr_batch_s *tsqr_batch;

/* Default row block and tree of the batched path when no table is given. */
#define TSQR_BATCH_DEFAULT_ROW_BLOCK 4096

/* Device workspace for a batch (only m, n, prec of the items are read).
   tune == NULL: the largest over the whole autotuning space, so the same
   workspace serves tsqr_autotune and any table it returns.  0 on error. */
TSQR_API size_t tsqr_batch_workspace_bytes(int count, const tsqr_batch_item *items,
                                           const tsqr_tune_entry *tune, int ntune);

/* Plans the batch (host), writes its device descriptors into dwork (256-byte
   aligned, >= tsqr_batch_workspace_bytes) on `stream`, and returns a host
   handle.  refine_sweeps: refinement sweeps after the first solve for the
   mixed matrices (each stops early on its own once its estimated remaining
   error (||dx|| times the observed contraction) is <= refine_tol ||x||
   or it stalls; the sweeps are part of the captured graph, so no host
   synchronisation happens inside a run).  Errors: -1 count, -2 items (an
   item out of scope: its index is reported by tsqr_batch_bad_item), -3 tune,
   -5 refine arguments, TSQR_ERR_WORKSPACE, -1000-e. */
TSQR_API int tsqr_batch_create(int count, const tsqr_batch_item *items, const tsqr_tune_entry *tune,
                               int ntune, int refine_sweeps, double refine_tol, void *dwork,
                               size_t work_bytes, void *stream, tsqr_batch *out);

/* Index of the first invalid item seen by the last failed
   tsqr_batch_create / tsqr_batch_workspace_bytes, or -1. */
TSQR_API int tsqr_batch_bad_item(void);

/* Runs the whole batch on `stream`.  use_graph = 1: the first call captures
   the launch sequence into a HIP graph bound to this handle (stream must
   not be NULL), later calls replay it; use_graph = 0: plain launches. */
TSQR_API int tsqr_batch_run(tsqr_batch b, int use_graph, void *stream);

/* Plan of item i (host): rows per domain, tree and number of domains. */
TSQR_API int tsqr_batch_plan(tsqr_batch b, int i, int64_t *row_block, int32_t *tree,
                             int64_t *domains);

/* Number of launches one run of the batch enqueues (graph nodes). */
TSQR_API int tsqr_batch_launches(tsqr_batch b);

TSQR_API int tsqr_batch_free(tsqr_batch b);

/* Autotuner: times the batch (plain launches, `reps` timed runs after one
   warm-up, HIP events on `stream`) over row_block in {512, 1024, 2048,
   4096, 8192} x tree in {binary, 4-ary, flat}: first one setting for all
   matrices, then each (n class, precision) class on its own with the others
   held at the best so far (its row block, then its tree; a change is kept
   when it saves at least 1 %).  n classes are n <= 8, 16, 32, 64.  Writes at
   most `cap` entries to out and returns the number written (< 0: error).
   dwork must hold tsqr_batch_workspace_bytes(count, items, NULL, 0); the
   items' outputs are overwritten. */
TSQR_API int tsqr_autotune(int count, const tsqr_batch_item *items, int reps, void *dwork,
                           size_t work_bytes, void *stream, tsqr_tune_entry *out, int cap);

/* ------------------------------------------------------------------------
   Serving: a request loop for least-squares solves of different sizes.
   Requests arrive with HOST matrices; the server admits them while its
   device memory budget and slot count allow (continuous batching: requests
   admitted while others run share the GPU through several HIP streams),
   copies A and B in, factors A (tsqr_factor) unless a factor of the same
   matrix is cached, solves (tsqr_lsq_solve) and copies X, the residual norms
   and info back.  Factors of finished requests stay cached (LRU) while the
   budget allows, so a repeated matrix costs only the solve.
   Allocation: tsqr_server_create allocates ONE device arena of hbm_budget
   bytes (hipMalloc) and creates the streams and events; everything else is
   carved from the arena.  tsqr_server_free releases them.  Host buffers
   should be pinned (hipHostMalloc) for the copies to overlap.
   Not thread-safe: one host thread drives a server.
   ------------------------------------------------------------------------ */
typedef struct tsqr_server_s *tsqr_server;

typedef struct {
    size_t hbm_budget;      /* device bytes of the arena                     */
    int32_t streams;        /* HIP streams (>= 1)                            */
    int32_t max_inflight;   /* requests admitted at once (>= 1)              */
    int32_t cache;          /* 1: keep factors of finished requests          */
    int32_t prec;           /* TSQR_F64 or TSQR_MIXED for every request      */
    int32_t tree;           /* TSQR_TREE_*                                   */
    int32_t bypass_ms;      /* a queued request whose memory does not fit   */
                            /* yet lets younger requests that fit be         */
                            /* admitted past it until it has waited this     */
                            /* long (ms); 0 = 100 ms, < 0 = strict FIFO       */
    int32_t reserved;
    double route_kappa;     /* TSQR_MIXED: a request whose R has a condition */
                            /* estimate above this is solved in FP64        */
                            /* (opts.route_kappa); default 1e4, 0 = never    */
} tsqr_server_opts;

typedef struct {
    int64_t matrix_id;      /* requests with equal ids share A (same m, n)   */
    int64_t m, n, k;        /* 1 <= n <= 256, n <= m, 1 <= k <= 8            */
    const double *A;        /* host, m x n column-major (lda = m); read at   */
                            /* admission unless the factor is cached         */
    const double *B;        /* host, m x k column-major (ldb = m)            */
    double *X;              /* host output, n x k (ldx = n)                  */
    double *resid;          /* host output, k residual norms                 */
    int32_t *info;          /* host output, tsqr_lsq_solve's dinfo           */
} tsqr_request;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t cache_hits, evictions;
    size_t bytes_in_use, bytes_peak;
    double busy_seconds;            /* time with >= 1 request admitted       */
    double byte_seconds;            /* integral of bytes in use over time    */
} tsqr_server_stats;

TSQR_API void tsqr_server_default_opts(tsqr_server_opts *o);
TSQR_API int tsqr_server_create(const tsqr_server_opts *o, tsqr_server *out);
/* Queues a request (the descriptor is copied; its host buffers must stay
   valid until the request is done).  Returns a ticket >= 0 or an error:
   -2 shape out of scope, -3 NULL buffer, -4 matrix_id reused with another
   shape, TSQR_ERR_WORKSPACE when it can never fit the budget. */
TSQR_API int64_t tsqr_server_submit(tsqr_server s, const tsqr_request *r);
/* Retires finished requests and admits queued ones in arrival order while
   slots are free.  A request that does not fit even after evicting idle
   cached factors waits; younger requests that fit are admitted past it
   until it has waited bypass_ms, after which nothing passes it.  A
   mixed-precision solve (which reads its convergence flag back after every
   refinement sweep) is enqueued by a worker thread of the server, so this
   call never waits for a refinement.  wait = 1 blocks until at least one
   request finishes when any is running.  Returns the number of requests
   queued or running. */
TSQR_API int tsqr_server_progress(tsqr_server s, int wait);
/* 1 when the request's outputs are written, 0 while pending, < 0 on error. */
TSQR_API int tsqr_server_status(tsqr_server s, int64_t ticket);
/* Steady-clock times (s) of submission, admission and completion. */
TSQR_API int tsqr_server_times(tsqr_server s, int64_t ticket, double *t_submit, double *t_admit,
                               double *t_done);
TSQR_API int tsqr_server_get_stats(tsqr_server s, tsqr_server_stats *st);
/* Finishes every request, then frees the arena, streams and handle. */
TSQR_API int tsqr_server_free(tsqr_server s);
/* Seconds on the server's steady clock (for arrival schedules). */
TSQR_API double tsqr_server_now(void);

/* Frees the host handle only (the workspace belongs to the caller). */
TSQR_API int tsqr_free(tsqr_factors f);

/* Static description of an error code. */
TSQR_API const char *tsqr_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_H_ */
