/*
 * tsqr_oracle.c -- plain FP64 CPU reference for TSQR.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product library never calls it, and the
 * two share no code, headers, tables or helpers.
 *
 * What it computes (Agullo, Coti, Dongarra, Herault, Langou, "QR
 * Factorization of Tall and Skinny Matrices in a Grid Computing Environment"):
 *   - Householder reflectors H = I - tau v v^T  (Sec. 2.2),
 *   - the compact-WY form H_1...H_b = I - V T V^T with T upper triangular
 *     (Sec. 2.2, Schreiber and Van Loan's accumulation),
 *   - TSQR (Sec. 2.3): the matrix is split into P block rows ("domains"),
 *     each domain gets a Householder QR, and the stacked R factors are
 *     reduced pairwise, R = qr([R_l; R_r]).R, up a binary, k-ary or flat
 *     tree.  The combine is associative, and commutative once the diagonal
 *     of every R is made nonnegative (Sec. 2.3), so R does not depend on
 *     the tree; that is the invariant the tests lean on,
 *   - uniqueness of R with a positive diagonal (Sec. 2.2), used here as the
 *     sign normalisation R <- D R, Q <- Q D with D = diag(sgn R_jj) and
 *     sgn(0) = +1,
 *   - applying Q^T, forming the thin Q, and least squares through the
 *     factors (the paper mentions QR as the first step toward least squares
 *     only in its draft text; the solve is the textbook one).
 *
 * Readings where the paper is silent:
 *   - reflector convention is LAPACK's: beta = -sgn(alpha) sqrt(alpha^2 +
 *     sigma^2), tau = (beta - alpha) / beta, v = [1; x / (alpha - beta)];
 *     tau = 0 when the subcolumn below alpha is exactly zero;
 *   - norms are plain sequential sums of squares, no scaling;
 *   - partition: P = ceil(m / mb) contiguous domains; a last domain with
 *     fewer than n rows is merged into the one before it;
 *   - load-balanced partition (Sec. 3 names it as future work): rows in
 *     whole granules, apportioned to the domains' integer powers by largest
 *     remainders, ties to the lower index;
 *   - tree results always land in the lower-index child, so the root is
 *     domain 0 and its first n rows are global rows 0..n-1;
 *   - binary tree: adjacent pairs per level, an odd node passes up;
 *     k-ary: groups of k consecutive live nodes, each reduced left to right;
 *     flat: R <- comb(R, R_i) for i = 1..P-1.
 *
 * Everything is plain loops in IEEE double, column-major storage.  Domains
 * are independent, so the leaf phase and the leaf part of apply/form-Q run
 * domains in parallel with OpenMP; nothing else is reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_API __attribute__((visibility("default")))


/* ------------------------------------------------------------------------ */
/* Householder reflector (Sec. 2.2: H = I - tau v v^T).                      */
/* In: *alpha = x_1, x[0..nx-1] = x_2 (stride incx).                         */
/* Out: *alpha = beta (H x = beta e_1), x = v_2 (v_1 = 1 implicit), *tau.    */
/* ------------------------------------------------------------------------ */
ORACLE_API void or_larfg(int64_t nx, double *alpha, double *x, int64_t incx, double *tau)
{
    double s2 = 0.0;
    for (int64_t i = 0; i < nx; ++i) s2 += x[i * incx] * x[i * incx];
    if (s2 == 0.0) {            /* nothing to annihilate: H = I */
        *tau = 0.0;
        return;
    }
    double a = *alpha;
    double sgn = (a < 0.0) ? -1.0 : 1.0;     /* sgn(0) = +1 */
    double beta = -sgn * sqrt(a * a + s2);
    *tau = (beta - a) / beta;
    double scal = 1.0 / (a - beta);
    for (int64_t i = 0; i < nx; ++i) x[i * incx] *= scal;
    *alpha = beta;
}

/* ------------------------------------------------------------------------ */
/* Leaf: Householder QR of an r x n block (Sec. 2.2, 2.3 "factorization of a */
/* domain").  On exit R is on and above the diagonal, v_j is below it (unit  */
/* diagonal implicit), tau[j] holds tau_j, and T (ldt >= n, may be NULL) is  */
/* the upper-triangular compact-WY factor with H_1...H_k = I - V T V^T.      */
/* k = min(r, n) reflectors are generated; for j >= k, tau_j = 0.            */
/* ------------------------------------------------------------------------ */
ORACLE_API void or_geqrt(int64_t r, int64_t n, double *A, int64_t lda, double *tau,
                         double *T, int64_t ldt)
{
    int64_t k = r < n ? r : n;
    for (int64_t j = 0; j < n; ++j) tau[j] = 0.0;
    for (int64_t j = 0; j < k; ++j) {
        double *col = A + j + j * lda;
        or_larfg(r - j - 1, col, col + 1, 1, &tau[j]);
        /* apply H_j to the trailing columns: a <- a - tau v (v^T a) */
        for (int64_t c = j + 1; c < n; ++c) {
            double *ac = A + j + c * lda;
            double w = ac[0];
            for (int64_t i = 1; i < r - j; ++i) w += col[i] * ac[i];
            w *= tau[j];
            ac[0] -= w;
            for (int64_t i = 1; i < r - j; ++i) ac[i] -= w * col[i];
        }
    }
    if (!T) return;
    /* T: T_jj = tau_j, T[0:j, j] = -tau_j T[0:j,0:j] (V[:,0:j]^T v_j). */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) T[i + j * ldt] = 0.0;
    for (int64_t j = 0; j < k; ++j) {
        double z[j > 0 ? j : 1];
        for (int64_t i = 0; i < j; ++i) {
            /* (V^T v_j)_i: v_j is 0 above row j, 1 at row j */
            double s = A[j + i * lda];
            for (int64_t q = j + 1; q < r; ++q) s += A[q + i * lda] * A[q + j * lda];
            z[i] = s;
        }
        for (int64_t i = 0; i < j; ++i) {
            double s = 0.0;
            for (int64_t q = i; q < j; ++q) s += T[i + q * ldt] * z[q];
            T[i + j * ldt] = -tau[j] * s;
        }
        T[j + j * ldt] = tau[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Tree combine (Sec. 2.3): QR of [R1; R2] with R1, R2 n x n upper           */
/* triangular (entries below the diagonal are ignored).  Reflector j is      */
/* [e_j; u_j] where u_j has nonzeros only in rows 0..j of the R2 block, so   */
/* the structural zeros stay zero.  On exit R1 holds R, the upper triangle   */
/* of R2 holds the u_j (column j, rows 0..j), tau[j], and T (may be NULL).   */
/* ------------------------------------------------------------------------ */
ORACLE_API void or_tpqrt(int64_t n, double *R1, int64_t ld1, double *R2, int64_t ld2,
                         double *tau, double *T, int64_t ldt)
{
    for (int64_t j = 0; j < n; ++j) {
        double *u = R2 + j * ld2;                    /* rows 0..j of column j */
        or_larfg(j + 1, &R1[j + j * ld1], u, 1, &tau[j]);
        for (int64_t c = j + 1; c < n; ++c) {
            double w = R1[j + c * ld1];
            for (int64_t i = 0; i <= j; ++i) w += u[i] * R2[i + c * ld2];
            w *= tau[j];
            R1[j + c * ld1] -= w;
            for (int64_t i = 0; i <= j; ++i) R2[i + c * ld2] -= w * u[i];
        }
    }
    if (!T) return;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) T[i + j * ldt] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double z[j > 0 ? j : 1];
        for (int64_t i = 0; i < j; ++i) {
            /* [e_i; u_i]^T [e_j; u_j] = u_i^T u_j (u_i lives in rows 0..i) */
            double s = 0.0;
            for (int64_t q = 0; q <= i; ++q) s += R2[q + i * ld2] * R2[q + j * ld2];
            z[i] = s;
        }
        for (int64_t i = 0; i < j; ++i) {
            double s = 0.0;
            for (int64_t q = i; q < j; ++q) s += T[i + q * ldt] * z[q];
            T[i + j * ldt] = -tau[j] * s;
        }
        T[j + j * ldt] = tau[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Partition into domains (Sec. 2.3 "P block-rows, called domains").         */
/* Returns P; fills row0/nrows when they are not NULL.                       */
/* ------------------------------------------------------------------------ */
ORACLE_API int64_t or_partition(int64_t m, int64_t n, int64_t mb, int64_t *row0, int64_t *nrows)
{
    if (mb < n || m < n || n < 1) return -1;
    int64_t P = (m + mb - 1) / mb;
    if (P > 1 && m - (P - 1) * mb < n) P -= 1;    /* merge a short last domain */
    if (row0 && nrows) {
        for (int64_t i = 0; i < P; ++i) {
            row0[i] = i * mb;
            nrows[i] = (i == P - 1) ? m - i * mb : mb;
        }
    }
    return P;
}

/* ------------------------------------------------------------------------ */
/* Load-balanced partition (Sec. 3: the rows given to each domain follow    */
/* the processing power dedicated to it).  w[d] >= 1 is the power of domain */
/* d in integer units (e.g. its cores; NULL = equal power).  Rows go out in */
/* whole granules of g rows, the last granule short when g does not divide */
/* m: C = ceil(m / g) granules, domain d first gets floor(C w_d / W) of     */
/* them (W = sum of w), and the C - sum floor(...) granules left over go    */
/* one each to the domains with the largest remainders C w_d mod W, ties    */
/* to the lower index (largest-remainder apportionment, exact in integers). */
/* Domains are contiguous in index order; the last one ends at row m.       */
/* Returns P, or -1 if some domain would hold no granule or fewer than n    */
/* rows.  Fills row0/nrows when they are not NULL.                          */
/* ------------------------------------------------------------------------ */
ORACLE_API int64_t or_partition_weighted(int64_t m, int64_t n, int64_t P, int64_t g,
                                         const int64_t *w, int64_t *row0, int64_t *nrows)
{
    if (m < n || n < 1 || P < 1 || g < 1) return -1;
    int64_t C = (m + g - 1) / g, W = 0;
    for (int64_t d = 0; d < P; ++d) {
        int64_t wd = w ? w[d] : 1;
        if (wd < 1 || wd > ((int64_t)1 << 31)) return -1;   /* C w_d stays in 64 bits */
        W += wd;
    }
    int64_t *k = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
    int64_t *rem = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
    int64_t given = 0;
    for (int64_t d = 0; d < P; ++d) {
        int64_t wd = w ? w[d] : 1;
        k[d] = C * wd / W;
        rem[d] = C * wd % W;
        given += k[d];
    }
    for (int64_t left = C - given; left > 0; --left) {
        int64_t best = -1;
        for (int64_t d = 0; d < P; ++d)
            if (rem[d] >= 0 && (best < 0 || rem[d] > rem[best])) best = d;
        k[best] += 1;
        rem[best] = -1;      /* one extra granule per domain at most */
    }
    int64_t ok = P, r = 0;
    for (int64_t d = 0; d < P; ++d) {
        int64_t rows = (d == P - 1) ? m - r : g * k[d];
        if (k[d] < 1 || rows < n) ok = -1;
        if (row0 && nrows) { row0[d] = r; nrows[d] = rows; }
        r += g * k[d];
    }
    free(k); free(rem);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Reduction-tree schedules (Sec. 2.3: binary, flat; k-ary generalises the  */
/* binary tree).  A schedule is an ordered list of combines (left, right);  */
/* the result stays in the left slot.  Returns the number of combines      */
/* (always P - 1).  tree: 0 = flat, 2 = binary, k >= 3 = k-ary.             */
/* ------------------------------------------------------------------------ */
ORACLE_API int64_t or_schedule(int64_t P, int tree, int64_t *sl, int64_t *sr)
{
    int64_t cnt = 0;
    if (tree == 0) {
        for (int64_t i = 1; i < P; ++i) { sl[cnt] = 0; sr[cnt] = i; ++cnt; }
        return cnt;
    }
    int k = tree < 2 ? 2 : tree;
    int64_t *live = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
    int64_t nl = P;
    for (int64_t i = 0; i < P; ++i) live[i] = i;
    while (nl > 1) {
        int64_t nn = 0;
        for (int64_t g = 0; g < nl; g += k) {
            int64_t end = g + k < nl ? g + k : nl;
            for (int64_t q = g + 1; q < end; ++q) { sl[cnt] = live[g]; sr[cnt] = live[q]; ++cnt; }
            live[nn++] = live[g];
        }
        nl = nn;
    }
    free(live);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* The factored object: leaf reflectors in place of a copy of A, per-domain */
/* tau/T, per-combine u/tau/T, and the sign-normalised R.                   */
/* ------------------------------------------------------------------------ */
typedef struct or_tsqr_s {
    int64_t m, n, P, nnodes;
    int64_t *row0, *nrows;
    double *W;              /* m x n, ld m: R on top of each domain, v below */
    double *tau;            /* P x n */
    double *T;              /* P x n x n */
    int64_t *sl, *sr;       /* schedule */
    double *U, *taun, *Tn;  /* nnodes x n x n, nnodes x n, nnodes x n x n */
    double *R;              /* n x n, sign-normalised */
    double *d;              /* n signs, D = diag(d) */
    int nthreads;
} or_tsqr;

ORACLE_API void or_free(or_tsqr *f)
{
    if (!f) return;
    free(f->row0); free(f->nrows); free(f->W); free(f->tau); free(f->T);
    free(f->sl); free(f->sr); free(f->U); free(f->taun); free(f->Tn);
    free(f->R); free(f->d); free(f);
}

/* Factor over an explicit partition (P contiguous domains covering rows  */
/* 0..m-1 in order, each of at least n rows) with an explicit schedule     */
/* (nnodes combines, result in the left).                                  */
ORACLE_API or_tsqr *or_factor_parts(int64_t m, int64_t n, const double *A, int64_t lda,
                                    int64_t P, const int64_t *row0, const int64_t *nrows,
                                    int64_t nnodes, const int64_t *sl, const int64_t *sr,
                                    int nthreads)
{
    if (P < 1 || n < 1 || lda < m || nnodes != P - 1) return NULL;
    for (int64_t i = 0, r = 0; i < P; r += nrows[i], ++i)
        if (row0[i] != r || nrows[i] < n || (i == P - 1 && r + nrows[i] != m)) return NULL;
    or_tsqr *f = (or_tsqr *)calloc(1, sizeof(or_tsqr));
    f->m = m; f->n = n; f->P = P; f->nnodes = nnodes;
    f->nthreads = nthreads > 0 ? nthreads : 1;
    f->row0 = (int64_t *)malloc(sizeof(int64_t) * P);
    f->nrows = (int64_t *)malloc(sizeof(int64_t) * P);
    for (int64_t i = 0; i < P; ++i) { f->row0[i] = row0[i]; f->nrows[i] = nrows[i]; }
    f->W = (double *)malloc(sizeof(double) * (size_t)m * n);
    for (int64_t c = 0; c < n; ++c)
        memcpy(f->W + c * m, A + c * lda, sizeof(double) * (size_t)m);
    f->tau = (double *)calloc((size_t)P * n, sizeof(double));
    f->T = (double *)calloc((size_t)P * n * n, sizeof(double));
    f->sl = (int64_t *)malloc(sizeof(int64_t) * (nnodes > 0 ? nnodes : 1));
    f->sr = (int64_t *)malloc(sizeof(int64_t) * (nnodes > 0 ? nnodes : 1));
    for (int64_t q = 0; q < nnodes; ++q) { f->sl[q] = sl[q]; f->sr[q] = sr[q]; }
    f->U = (double *)calloc((size_t)(nnodes > 0 ? nnodes : 1) * n * n, sizeof(double));
    f->taun = (double *)calloc((size_t)(nnodes > 0 ? nnodes : 1) * n, sizeof(double));
    f->Tn = (double *)calloc((size_t)(nnodes > 0 ? nnodes : 1) * n * n, sizeof(double));
    f->R = (double *)calloc((size_t)n * n, sizeof(double));
    f->d = (double *)malloc(sizeof(double) * n);

    /* leaves: one Householder QR per domain */
#pragma omp parallel for schedule(dynamic) num_threads(f->nthreads)
    for (int64_t i = 0; i < P; ++i)
        or_geqrt(f->nrows[i], n, f->W + f->row0[i], m, f->tau + i * n, f->T + i * n * n, n);

    /* the R of every live slot: n x n upper triangle copied out of W */
    double *Rs = (double *)calloc((size_t)P * n * n, sizeof(double));
    for (int64_t i = 0; i < P; ++i)
        for (int64_t c = 0; c < n; ++c)
            for (int64_t r = 0; r <= c; ++r)
                Rs[i * n * n + r + c * n] = f->W[f->row0[i] + r + c * m];

    /* tree: combines in schedule order */
    for (int64_t q = 0; q < nnodes; ++q) {
        double *Rl = Rs + f->sl[q] * n * n, *Rr = Rs + f->sr[q] * n * n;
        double *Uq = f->U + q * n * n;
        for (int64_t c = 0; c < n; ++c)
            for (int64_t r = 0; r <= c; ++r) Uq[r + c * n] = Rr[r + c * n];
        or_tpqrt(n, Rl, n, Uq, n, f->taun + q * n, f->Tn + q * n * n, n);
    }
    /* sign normalisation of the root (slot 0) */
    for (int64_t j = 0; j < n; ++j) f->d[j] = (Rs[j + j * n] < 0.0) ? -1.0 : 1.0;
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r <= c; ++r) f->R[r + c * n] = f->d[r] * Rs[r + c * n];
    free(Rs);
    return f;
}

/* Factor with the mb partition and an explicit schedule. */
ORACLE_API or_tsqr *or_factor_sched(int64_t m, int64_t n, const double *A, int64_t lda,
                                    int64_t mb, int64_t nnodes, const int64_t *sl,
                                    const int64_t *sr, int nthreads)
{
    int64_t P = or_partition(m, n, mb, NULL, NULL);
    if (P < 1) return NULL;
    int64_t *row0 = (int64_t *)malloc(sizeof(int64_t) * P);
    int64_t *nrows = (int64_t *)malloc(sizeof(int64_t) * P);
    or_partition(m, n, mb, row0, nrows);
    or_tsqr *f = or_factor_parts(m, n, A, lda, P, row0, nrows, nnodes, sl, sr, nthreads);
    free(row0); free(nrows);
    return f;
}

ORACLE_API or_tsqr *or_factor(int64_t m, int64_t n, const double *A, int64_t lda, int64_t mb,
                              int tree, int nthreads)
{
    int64_t P = or_partition(m, n, mb, NULL, NULL);
    if (P < 1) return NULL;
    int64_t *sl = (int64_t *)malloc(sizeof(int64_t) * (P > 1 ? P - 1 : 1));
    int64_t *sr = (int64_t *)malloc(sizeof(int64_t) * (P > 1 ? P - 1 : 1));
    int64_t nn = or_schedule(P, tree, sl, sr);
    or_tsqr *f = or_factor_sched(m, n, A, lda, mb, nn, sl, sr, nthreads);
    free(sl); free(sr);
    return f;
}

ORACLE_API int64_t or_num_domains(const or_tsqr *f) { return f->P; }

/* Sign-normalised R (n x n, upper triangular, zeros below). */
ORACLE_API void or_get_r(const or_tsqr *f, double *R, int64_t ldr)
{
    int64_t n = f->n;
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < n; ++r) R[r + c * ldr] = (r <= c) ? f->R[r + c * n] : 0.0;
}

/* Raw per-domain leaf output: W (m x n), tau (P x n), T (P x n x n). */
ORACLE_API void or_get_leaf(const or_tsqr *f, double *W, double *tau, double *T)
{
    if (W) memcpy(W, f->W, sizeof(double) * (size_t)f->m * f->n);
    if (tau) memcpy(tau, f->tau, sizeof(double) * (size_t)f->P * f->n);
    if (T) memcpy(T, f->T, sizeof(double) * (size_t)f->P * f->n * f->n);
}

/* ------------------------------------------------------------------------ */
/* B <- Q^T B (k columns, in place).  Leaves first (H_1 applied first), then */
/* the tree bottom-up in schedule order; finally the root rows are scaled by */
/* D so that rows 0..n-1 equal (Q_1 D)^T B for the sign-normalised Q_1.      */
/* ------------------------------------------------------------------------ */
ORACLE_API void or_apply_qt(const or_tsqr *f, int64_t k, double *B, int64_t ldb)
{
    int64_t m = f->m, n = f->n;
#pragma omp parallel for schedule(dynamic) num_threads(f->nthreads)
    for (int64_t i = 0; i < f->P; ++i) {
        const double *Wi = f->W + f->row0[i];
        int64_t r = f->nrows[i];
        int64_t kr = r < n ? r : n;
        for (int64_t j = 0; j < kr; ++j) {
            double t = f->tau[i * n + j];
            for (int64_t c = 0; c < k; ++c) {
                double *b = B + f->row0[i] + c * ldb;
                double w = b[j];
                for (int64_t q = j + 1; q < r; ++q) w += Wi[q + j * m] * b[q];
                w *= t;
                b[j] -= w;
                for (int64_t q = j + 1; q < r; ++q) b[q] -= w * Wi[q + j * m];
            }
        }
    }
    for (int64_t q = 0; q < f->nnodes; ++q) {
        const double *Uq = f->U + q * n * n;
        const double *tq = f->taun + q * n;
        for (int64_t c = 0; c < k; ++c) {
            double *yl = B + f->row0[f->sl[q]] + c * ldb;
            double *yr = B + f->row0[f->sr[q]] + c * ldb;
            for (int64_t j = 0; j < n; ++j) {
                double w = yl[j];
                for (int64_t i = 0; i <= j; ++i) w += Uq[i + j * n] * yr[i];
                w *= tq[j];
                yl[j] -= w;
                for (int64_t i = 0; i <= j; ++i) yr[i] -= w * Uq[i + j * n];
            }
        }
    }
    for (int64_t c = 0; c < k; ++c)
        for (int64_t j = 0; j < n; ++j) B[j + c * ldb] *= f->d[j];
    (void)m;
}

/* ------------------------------------------------------------------------ */
/* Thin Q (m x n), sign-normalised so that A = Q R with diag(R) >= 0.       */
/* Start from [D; 0] at the root, apply the tree top-down (reverse schedule,*/
/* H_n first at each node), then each leaf (H_n first).                     */
/* ------------------------------------------------------------------------ */
ORACLE_API void or_form_q(const or_tsqr *f, double *Q, int64_t ldq)
{
    int64_t m = f->m, n = f->n;
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < m; ++r) Q[r + c * ldq] = 0.0;
    for (int64_t j = 0; j < n; ++j) Q[j + j * ldq] = f->d[j];
    for (int64_t q = f->nnodes - 1; q >= 0; --q) {
        const double *Uq = f->U + q * n * n;
        const double *tq = f->taun + q * n;
        for (int64_t c = 0; c < n; ++c) {
            double *yl = Q + f->row0[f->sl[q]] + c * ldq;
            double *yr = Q + f->row0[f->sr[q]] + c * ldq;
            for (int64_t j = n - 1; j >= 0; --j) {
                double w = yl[j];
                for (int64_t i = 0; i <= j; ++i) w += Uq[i + j * n] * yr[i];
                w *= tq[j];
                yl[j] -= w;
                for (int64_t i = 0; i <= j; ++i) yr[i] -= w * Uq[i + j * n];
            }
        }
    }
#pragma omp parallel for schedule(dynamic) num_threads(f->nthreads)
    for (int64_t i = 0; i < f->P; ++i) {
        const double *Wi = f->W + f->row0[i];
        int64_t r = f->nrows[i];
        int64_t kr = r < n ? r : n;
        for (int64_t j = kr - 1; j >= 0; --j) {
            double t = f->tau[i * n + j];
            for (int64_t c = 0; c < n; ++c) {
                double *b = Q + f->row0[i] + c * ldq;
                double w = b[j];
                for (int64_t q = j + 1; q < r; ++q) w += Wi[q + j * m] * b[q];
                w *= t;
                b[j] -= w;
                for (int64_t q = j + 1; q < r; ++q) b[q] -= w * Wi[q + j * m];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Least squares min ||A x - b|| for k right-hand sides through the factors:*/
/* C = Q^T B; X = R^{-1} C[0:n] by back substitution; resid_c = ||C[n:m,c]||.*/
/* Returns 0, or j+1 for the first exactly-zero R_jj (X not written).       */
/* ------------------------------------------------------------------------ */
ORACLE_API int64_t or_lsq(const or_tsqr *f, int64_t k, const double *B, int64_t ldb,
                          double *X, int64_t ldx, double *resid)
{
    int64_t m = f->m, n = f->n;
    for (int64_t j = 0; j < n; ++j)
        if (f->R[j + j * n] == 0.0) return j + 1;
    double *C = (double *)malloc(sizeof(double) * (size_t)m * k);
    for (int64_t c = 0; c < k; ++c)
        memcpy(C + c * m, B + c * ldb, sizeof(double) * (size_t)m);
    or_apply_qt(f, k, C, m);
    for (int64_t c = 0; c < k; ++c) {
        double *cc = C + c * m;
        for (int64_t j = n - 1; j >= 0; --j) {
            double s = cc[j];
            for (int64_t q = j + 1; q < n; ++q) s -= f->R[j + q * n] * X[q + c * ldx];
            X[j + c * ldx] = s / f->R[j + j * n];
        }
        if (resid) {
            double s = 0.0;
            for (int64_t r = n; r < m; ++r) s += cc[r] * cc[r];
            resid[c] = sqrt(s);
        }
    }
    free(C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Refined least-squares reference (tests only).  Bjorck's iterative        */
/* refinement of the augmented system [I A; A^T 0][r; x] = [b; 0] with the  */
/* residuals f = b - r - A x and g = -A^T r accumulated in binary128, and   */
/* the corrections solved through the FP64 factors:                        */
/*   R^T h = g,  d = Q^T f,  dx = R^{-1}(d_1 - h),  dr = Q [h; d_2].         */
/* Starts from x = R^{-1} Q_1^T b, r = b - A x, and stops when ||dx|| <=    */
/* 1e-17 ||x|| or after maxit sweeps.  One right-hand side.  Returns the    */
/* number of sweeps, or -1 when R is singular.                              */
/* ------------------------------------------------------------------------ */
static void or_apply_q_full(const or_tsqr *f, double *y)
{
    /* y (m) <- Q y for the full (unnormalised) orthogonal Q of the factors,
       where the root's first n entries are taken in the normalised basis.  */
    int64_t m = f->m, n = f->n;
    for (int64_t j = 0; j < n; ++j) y[j] *= f->d[j];
    for (int64_t q = f->nnodes - 1; q >= 0; --q) {
        const double *Uq = f->U + q * n * n;
        const double *tq = f->taun + q * n;
        double *yl = y + f->row0[f->sl[q]];
        double *yr = y + f->row0[f->sr[q]];
        for (int64_t j = n - 1; j >= 0; --j) {
            double w = yl[j];
            for (int64_t i = 0; i <= j; ++i) w += Uq[i + j * n] * yr[i];
            w *= tq[j];
            yl[j] -= w;
            for (int64_t i = 0; i <= j; ++i) yr[i] -= w * Uq[i + j * n];
        }
    }
    for (int64_t i = 0; i < f->P; ++i) {
        const double *Wi = f->W + f->row0[i];
        double *b = y + f->row0[i];
        int64_t r = f->nrows[i];
        int64_t kr = r < n ? r : n;
        for (int64_t j = kr - 1; j >= 0; --j) {
            double w = b[j];
            for (int64_t q = j + 1; q < r; ++q) w += Wi[q + j * m] * b[q];
            w *= f->tau[i * n + j];
            b[j] -= w;
            for (int64_t q = j + 1; q < r; ++q) b[q] -= w * Wi[q + j * m];
        }
    }
}

ORACLE_API int64_t or_lsq_refined(const or_tsqr *f, const double *A, int64_t lda,
                                  const double *b, double *x, int maxit)
{
    int64_t m = f->m, n = f->n;
    for (int64_t j = 0; j < n; ++j)
        if (f->R[j + j * n] == 0.0) return -1;
    double *r = (double *)malloc(sizeof(double) * m);
    double *fv = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * n);
    double *h = (double *)malloc(sizeof(double) * n);
    double *dx = (double *)malloc(sizeof(double) * n);
    const double *Rm = f->R;
    /* initial x and r */
    or_lsq(f, 1, b, m, x, n, NULL);
    for (int64_t i = 0; i < m; ++i) {
        __float128 s = b[i];
        for (int64_t j = 0; j < n; ++j) s -= (__float128)A[i + j * lda] * x[j];
        r[i] = (double)s;
    }
    int it;
    double nd_prev = -1.0;
    for (it = 0; it < maxit; ++it) {
        /* residuals in binary128 */
        for (int64_t i = 0; i < m; ++i) {
            __float128 s = (__float128)b[i] - r[i];
            for (int64_t j = 0; j < n; ++j) s -= (__float128)A[i + j * lda] * x[j];
            fv[i] = (double)s;
        }
        for (int64_t j = 0; j < n; ++j) {
            __float128 s = 0;
            for (int64_t i = 0; i < m; ++i) s -= (__float128)A[i + j * lda] * r[i];
            g[j] = (double)s;
        }
        /* R^T h = g (forward substitution) */
        for (int64_t j = 0; j < n; ++j) {
            double s = g[j];
            for (int64_t q = 0; q < j; ++q) s -= Rm[q + j * n] * h[q];
            h[j] = s / Rm[j + j * n];
        }
        or_apply_qt(f, 1, fv, m);              /* fv <- Q^T f = [d1; d2] */
        for (int64_t j = n - 1; j >= 0; --j) { /* dx = R^{-1}(d1 - h) */
            double s = fv[j] - h[j];
            for (int64_t q = j + 1; q < n; ++q) s -= Rm[j + q * n] * dx[q];
            dx[j] = s / Rm[j + j * n];
        }
        for (int64_t j = 0; j < n; ++j) fv[j] = h[j];
        or_apply_q_full(f, fv);                /* dr = Q [h; d2] */
        double nx = 0.0, nd = 0.0;
        for (int64_t j = 0; j < n; ++j) { x[j] += dx[j]; nx += x[j] * x[j]; nd += dx[j] * dx[j]; }
        for (int64_t i = 0; i < m; ++i) r[i] += fv[i];
        /* converged, or no longer contracting (x is then exact to within
           the rounding of its own FP64 representation) */
        if (nd <= 1e-34 * nx || (nd_prev >= 0.0 && nd > 0.25 * nd_prev)) { ++it; break; }
        nd_prev = nd;
    }
    free(r); free(fv); free(g); free(h); free(dx);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Condition of R in the 1-norm, kappa_1(R) = ||R||_1 ||R^{-1}||_1, for     */
/* routing ill-conditioned mixed-precision problems to FP64 (the paper is  */
/* FP64 only; this is the definition, written out).  R: n x n upper         */
/* triangular, column-major.  R^{-1} is formed column by column by back     */
/* substitution on the unit vectors.  Returns +inf for a zero diagonal.     */
/* ------------------------------------------------------------------------ */
static double or_norm1_tri(int64_t n, const double *R, int64_t ldr)
{
    double best = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i <= j; ++i) s += fabs(R[i + j * ldr]);
        if (s > best) best = s;
    }
    return best;
}

/* y <- R^{-1} y (back substitution). */
static void or_solve_r(int64_t n, const double *R, int64_t ldr, double *y)
{
    for (int64_t j = n - 1; j >= 0; --j) {
        y[j] /= R[j + j * ldr];
        for (int64_t i = 0; i < j; ++i) y[i] -= R[i + j * ldr] * y[j];
    }
}

/* y <- R^{-T} y (forward substitution with the transpose). */
static void or_solve_rt(int64_t n, const double *R, int64_t ldr, double *y)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < j; ++i) y[j] -= R[i + j * ldr] * y[i];
        y[j] /= R[j + j * ldr];
    }
}

ORACLE_API double or_cond1(int64_t n, const double *R, int64_t ldr)
{
    for (int64_t j = 0; j < n; ++j)
        if (R[j + j * ldr] == 0.0) return INFINITY;
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    double inv = 0.0;
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = 0; i < n; ++i) e[i] = (i == c) ? 1.0 : 0.0;
        or_solve_r(n, R, ldr, e);
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += fabs(e[i]);
        if (s > inv) inv = s;
    }
    free(e);
    return or_norm1_tri(n, R, ldr) * inv;
}

/* ------------------------------------------------------------------------ */
/* The cheap estimate of kappa_1(R): ||R||_1 times a lower bound on         */
/* ||R^{-1}||_1 from Hager's method (1984) with Higham's refinements (1988: */
/* at most five iterations, stop when the sign vector repeats or the       */
/* estimate stops growing, then compare with the alternating-sign vector   */
/* x_i = (-1)^i (1 + i / (n - 1)), i = 0..n-1, divided by its 1-norm 3n/2). */
/* Each iteration costs one solve with R and one with R^T.  Ties in the    */
/* argmax go to the lower index; sgn(0) = +1.  Returns +inf for a zero     */
/* diagonal.                                                               */
/* ------------------------------------------------------------------------ */
ORACLE_API double or_cond1_est(int64_t n, const double *R, int64_t ldr)
{
    for (int64_t j = 0; j < n; ++j)
        if (R[j + j * ldr] == 0.0) return INFINITY;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *xi = (double *)malloc(sizeof(double) * (size_t)n);
    double est;
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
    or_solve_r(n, R, ldr, x);
    if (n == 1) {
        est = fabs(x[0]);
    } else {
        est = 0.0;
        for (int64_t i = 0; i < n; ++i) { est += fabs(x[i]); xi[i] = x[i] >= 0.0 ? 1.0 : -1.0; }
        for (int64_t i = 0; i < n; ++i) x[i] = xi[i];
        or_solve_rt(n, R, ldr, x);
        int64_t j = 0;
        for (int64_t i = 1; i < n; ++i) if (fabs(x[i]) > fabs(x[j])) j = i;
        for (int iter = 2; iter <= 5; ++iter) {
            for (int64_t i = 0; i < n; ++i) x[i] = (i == j) ? 1.0 : 0.0;
            or_solve_r(n, R, ldr, x);
            double old = est, nrm = 0.0;
            int same = 1;
            for (int64_t i = 0; i < n; ++i) {
                nrm += fabs(x[i]);
                double sg = x[i] >= 0.0 ? 1.0 : -1.0;
                if (sg != xi[i]) same = 0;
                xi[i] = sg;
            }
            est = nrm;
            if (same || est <= old) { if (est < old) est = old; break; }
            for (int64_t i = 0; i < n; ++i) x[i] = xi[i];
            or_solve_rt(n, R, ldr, x);
            int64_t jl = j;
            j = 0;
            for (int64_t i = 1; i < n; ++i) if (fabs(x[i]) > fabs(x[j])) j = i;
            if (fabs(x[jl]) == fabs(x[j])) break;
        }
        for (int64_t i = 0; i < n; ++i)
            x[i] = ((i % 2) ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1));
        or_solve_r(n, R, ldr, x);
        double t = 0.0;
        for (int64_t i = 0; i < n; ++i) t += fabs(x[i]);
        t = 2.0 * t / (3.0 * (double)n);
        if (t > est) est = t;
    }
    free(x); free(xi);
    return or_norm1_tri(n, R, ldr) * est;
}

/* ------------------------------------------------------------------------ */
/* TSLU: LU of a tall-skinny matrix with tournament pivoting, the extension */
/* the paper names in its conclusion (TSQR's reduction tree carries over  */
/* to LU, CALU's panel factorization).  The tree selects b pivot rows:     */
/*   - a node takes a stack of original rows of A (its children's selected */
/*     rows, or raw rows of A) and runs Gaussian elimination with partial  */
/*     pivoting on it; the b rows chosen as pivots, in order, are its      */
/*     selection (the original rows, not their eliminated values);        */
/*   - inside a domain the rows are taken in stages, a flat tree: the first */
/*     `first` rows, then repeatedly the current selection stacked on the  */
/*     next `stage` rows;                                                  */
/*   - across domains the selections are combined along the schedule       */
/*     (left, right): the left's selection stacked on the right's.         */
/* The root's selection gives ipiv (global row indices, pivot order).  U    */
/* and the unit lower L11 are the LU factors of A[ipiv, :] without further */
/* pivoting, and every other row i gets l_i = a_i U^{-1}, so A = L U with  */
/* L (m x b) in A's row order (rows ipiv[k] hold L11's rows).  Ties in a  */
/* pivot search go to the lowest stack position (stacks keep their order, */
/* no rows are swapped); a zero pivot column takes its first active row,  */
/* eliminates nothing, and the solve for l_i leaves l_k = 0 where U_kk = 0.*/
/* Returns 0, j + 1 for the first U_jj = 0, or -1 for bad arguments.      */
/* ------------------------------------------------------------------------ */

/* Partial-pivoting elimination on the r x b stack S (column-major, ld r,  */
/* overwritten); sel receives the stack positions of the min(b, r) pivots. */
static void or_gepp_select(int64_t r, int64_t b, double *S, int64_t *sel)
{
    char *act = (char *)malloc((size_t)r);
    for (int64_t i = 0; i < r; ++i) act[i] = 1;
    int64_t kb = b < r ? b : r;
    for (int64_t j = 0; j < kb; ++j) {
        int64_t p = -1;
        double best = -1.0;
        for (int64_t i = 0; i < r; ++i)
            if (act[i] && fabs(S[i + j * r]) > best) { best = fabs(S[i + j * r]); p = i; }
        if (p < 0)   /* a column of NaNs: its first active row */
            for (int64_t i = r - 1; i >= 0; --i) if (act[i]) p = i;
        if (p < 0) break;    /* not reached: r - j >= 1 rows are active */
        sel[j] = p;
        act[p] = 0;
        double piv = S[p + j * r];
        if (piv == 0.0) continue;
        for (int64_t i = 0; i < r; ++i) {
            if (!act[i]) continue;
            double l = S[i + j * r] / piv;
            S[i + j * r] = l;
            for (int64_t k = j + 1; k < b; ++k) S[i + k * r] -= l * S[p + k * r];
        }
    }
    free(act);
}

/* Selection of the stack made of the rows idx[0..r-1] of A. */
static int64_t or_select_rows(int64_t b, const double *A, int64_t lda, int64_t r, const int64_t *idx,
                              int64_t *out)
{
    double *S = (double *)malloc(sizeof(double) * (size_t)r * b);
    int64_t *sel = (int64_t *)malloc(sizeof(int64_t) * (size_t)b);
    for (int64_t k = 0; k < b; ++k)
        for (int64_t i = 0; i < r; ++i) S[i + k * r] = A[idx[i] + k * lda];
    or_gepp_select(r, b, S, sel);
    int64_t kb = b < r ? b : r;
    for (int64_t j = 0; j < kb; ++j) out[j] = idx[sel[j]];
    free(S); free(sel);
    return kb;
}

ORACLE_API int64_t or_tslu(int64_t m, int64_t b, const double *A, int64_t lda, int64_t P,
                           const int64_t *row0, const int64_t *nrows, int64_t first, int64_t stage,
                           int64_t nnodes, const int64_t *sl, const int64_t *sr, int nthreads,
                           int64_t *ipiv, double *L, int64_t ldl, double *U, int64_t ldu)
{
    if (b < 1 || m < b || lda < m || ldl < m || ldu < b || P < 1 || first < b || stage < 1 ||
        nnodes != P - 1)
        return -1;
    for (int64_t d = 0, r = 0; d < P; r += nrows[d], ++d)
        if (row0[d] != r || nrows[d] < b || (d == P - 1 && r + nrows[d] != m)) return -1;
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)P * b);
    int nt = nthreads > 0 ? nthreads : 1;
    (void)nt;
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int64_t d = 0; d < P; ++d) {
        int64_t *cur = cand + d * b;
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(b + (first > stage ? first : stage)));
        int64_t end = row0[d] + nrows[d];
        int64_t pos = row0[d], nc = 0, r = 0;
        int64_t take = nrows[d] < first ? nrows[d] : first;
        for (int64_t i = 0; i < take; ++i) idx[r++] = pos + i;
        pos += take;
        nc = or_select_rows(b, A, lda, r, idx, cur);
        while (pos < end) {
            take = end - pos < stage ? end - pos : stage;
            r = 0;
            for (int64_t i = 0; i < nc; ++i) idx[r++] = cur[i];
            for (int64_t i = 0; i < take; ++i) idx[r++] = pos + i;
            pos += take;
            nc = or_select_rows(b, A, lda, r, idx, cur);
        }
        free(idx);
    }
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)2 * b);
    for (int64_t q = 0; q < nnodes; ++q) {
        for (int64_t i = 0; i < b; ++i) { idx[i] = cand[sl[q] * b + i]; idx[b + i] = cand[sr[q] * b + i]; }
        or_select_rows(b, A, lda, 2 * b, idx, cand + sl[q] * b);
    }
    free(idx);
    for (int64_t k = 0; k < b; ++k) ipiv[k] = cand[k];
    free(cand);

    /* U and L11: LU of A[ipiv, :] without pivoting */
    double *M = (double *)malloc(sizeof(double) * (size_t)b * b);
    for (int64_t k = 0; k < b; ++k)
        for (int64_t i = 0; i < b; ++i) M[i + k * b] = A[ipiv[i] + k * lda];
    int64_t info = 0;
    for (int64_t j = 0; j < b; ++j) {
        double piv = M[j + j * b];
        if (piv == 0.0) { if (!info) info = j + 1; continue; }
        for (int64_t i = j + 1; i < b; ++i) {
            double l = M[i + j * b] / piv;
            M[i + j * b] = l;
            for (int64_t k = j + 1; k < b; ++k) M[i + k * b] -= l * M[j + k * b];
        }
    }
    for (int64_t k = 0; k < b; ++k)
        for (int64_t i = 0; i < b; ++i) U[i + k * ldu] = (i <= k) ? M[i + k * b] : 0.0;
    /* L: the pivot rows from L11, every other row by l U = a */
    char *isp = (char *)calloc((size_t)m, 1);
    for (int64_t k = 0; k < b; ++k) isp[ipiv[k]] = 1;
    for (int64_t k = 0; k < b; ++k)
        for (int64_t i = 0; i < m; ++i) L[i + k * ldl] = 0.0;
    for (int64_t i = 0; i < b; ++i)
        for (int64_t k = 0; k < b; ++k)
            L[ipiv[i] + k * ldl] = (k < i) ? M[i + k * b] : (k == i ? 1.0 : 0.0);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < m; ++i) {
        if (isp[i]) continue;
        for (int64_t k = 0; k < b; ++k) {
            double s = A[i + k * lda];
            for (int64_t j = 0; j < k; ++j) s -= L[i + j * ldl] * U[j + k * ldu];
            L[i + k * ldl] = (U[k + k * ldu] == 0.0) ? 0.0 : s / U[k + k * ldu];
        }
    }
    free(isp); free(M);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Cholesky factorization A = L L^T of a symmetric positive definite n x n  */
/* matrix, the third one-sided factorization the paper's introduction and   */
/* conclusion name beside QR and LU.  This is the definition written out    */
/* column by column (Cholesky-Crout order):                                 */
/*   l_jj = sqrt(a_jj - sum_{k<j} l_jk^2),                                  */
/*   l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj   for i > j,                */
/* each sum taken in increasing k.  Only the lower triangle of A is read.   */
/* L (ldl >= n) receives L with zeros above the diagonal.  Returns 0, or     */
/* j + 1 when the leading minor of order j + 1 is not positive definite     */
/* (a_jj - sum <= 0 or NaN): columns 0..j-1 of L are then final and the     */
/* rest are zero.  The rows of a column are independent and run in         */
/* parallel with OpenMP; L is kept row by row inside so the sums read       */
/* consecutive memory.                                                      */
/* ------------------------------------------------------------------------ */
ORACLE_API int64_t or_cholesky(int64_t n, const double *A, int64_t lda, double *L, int64_t ldl, int nthreads)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || ldl < (n > 1 ? n : 1)) return -1;
    const int nt = nthreads > 0 ? nthreads : 1;
    double *Lr = (double *)calloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1), sizeof(double));
    int64_t info = 0;
    for (int64_t j = 0; j < n && !info; ++j) {
        const double *lj = Lr + j * n;
        double d = A[j + j * lda];
        for (int64_t k = 0; k < j; ++k) d -= lj[k] * lj[k];
        if (!(d > 0.0)) { info = j + 1; break; }
        const double ljj = sqrt(d);
        Lr[j * n + j] = ljj;
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = j + 1; i < n; ++i) {
            const double *li = Lr + i * n;
            double s = A[i + j * lda];
            for (int64_t k = 0; k < j; ++k) s -= li[k] * lj[k];
            Lr[i * n + j] = s / ljj;
        }
    }
    const int64_t done = info ? info - 1 : n;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            L[i + j * ldl] = (i >= j && j < done) ? Lr[i * n + j] : 0.0;
    free(Lr);
    return info;
}

/* ------------------------------------------------------------------------ */
/* CALU: LU of an m x n matrix (m >= n) with tournament pivoting, the LU    */
/* counterpart of CAQR that the conclusion names beside TSLU.  Panels of    */
/* b = 64 columns (the last one narrower); panel k:                         */
/*   1. TSLU (or_tslu) of the m - k rows below the diagonal, over the       */
/*      domains of or_partition(m - k, b, mb) and the or_schedule tree,     */
/*      stacks of 256 rows;                                                 */
/*   2. the tournament's pivot rows become b row interchanges in LAPACK's   */
/*      style: interchange i swaps rows k + i and k + swp[i], where swp[i]  */
/*      is where the i-th pivot row sits after interchanges 0..i-1;         */
/*      ipiv[k + i] = k + swp[i];                                           */
/*   3. the interchanges are applied to every column outside the panel, and */
/*      the panel's columns take L and U in the permuted row order (U in    */
/*      and above the diagonal block's diagonal, the unit lower L11 below   */
/*      it, L21 under the block);                                           */
/*   4. U12 = L11^{-1} A12 (forward substitution, unit diagonal) and        */
/*      A22 -= L21 U12.                                                     */
/* A is overwritten LAPACK-style (dgetrf's packed L\U).  Returns 0, or the  */
/* first k + j + 1 whose U_jj is exactly zero (that column's l entries are  */
/* zero and the factorization goes on), or -1 on bad arguments.             */
/* ------------------------------------------------------------------------ */
ORACLE_API int64_t or_calu(int64_t m, int64_t n, double *A, int64_t lda, int64_t mb, int tree, int nthreads,
                           int64_t *ipiv)
{
    if (n < 1 || m < n || lda < m || mb < 1) return -1;
    const int64_t bw = 64;
    int64_t info = 0;
    int64_t *row0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *nrows = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *sl = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *sr = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *rowat = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *posof = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    double *Lp = (double *)malloc(sizeof(double) * (size_t)m * (size_t)bw);
    double *Up = (double *)malloc(sizeof(double) * (size_t)bw * (size_t)bw);
    int64_t piv[64], swp[64];
    for (int64_t k = 0; k < n; k += bw) {
        const int64_t b = (n - k < bw) ? n - k : bw;
        const int64_t mr = m - k;
        /* 1. the panel's tournament */
        const int64_t P = or_partition(mr, b, mb, row0, nrows);
        const int64_t nn = or_schedule(P, tree, sl, sr);
        const int64_t ik = or_tslu(mr, b, A + k + k * lda, lda, P, row0, nrows, 256, 256 - b, nn, sl, sr,
                                   nthreads, piv, Lp, mr, Up, b);
        if (ik > 0 && !info) info = k + ik;
        /* 2. pivot rows -> interchanges */
        for (int64_t r = 0; r < mr; ++r) { rowat[r] = r; posof[r] = r; }
        for (int64_t i = 0; i < b; ++i) {
            const int64_t r = piv[i], p = posof[r], ri = rowat[i];
            swp[i] = p;
            rowat[i] = r; rowat[p] = ri;
            posof[r] = i; posof[ri] = p;
            ipiv[k + i] = k + p;
        }
        /* 3. interchanges outside the panel; the panel's L and U */
        for (int64_t c = 0; c < n; ++c) {
            if (c >= k && c < k + b) continue;
            double *col = A + c * lda + k;
            for (int64_t i = 0; i < b; ++i) {
                const double t = col[i];
                col[i] = col[swp[i]];
                col[swp[i]] = t;
            }
        }
        for (int64_t j = 0; j < b; ++j)
            for (int64_t rel = 0; rel < mr; ++rel)
                A[k + rel + (k + j) * lda] = (rel < b && j >= rel) ? Up[rel + j * b] : Lp[rowat[rel] + j * mr];
        /* 4. U12 and the trailing update */
        for (int64_t c = k + b; c < n; ++c) {
            double *col = A + c * lda;
            for (int64_t i = 0; i < b; ++i) {
                double t = col[k + i];
                for (int64_t l = 0; l < i; ++l) t -= A[k + i + (k + l) * lda] * col[k + l];
                col[k + i] = t;
            }
        }
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
        for (int64_t c = k + b; c < n; ++c) {
            double *col = A + c * lda;
            for (int64_t i = k + b; i < m; ++i) {
                double t = col[i];
                for (int64_t l = 0; l < b; ++l) t -= A[i + (k + l) * lda] * col[k + l];
                col[i] = t;
            }
        }
    }
    free(row0); free(nrows); free(sl); free(sr); free(rowat); free(posof); free(Lp); free(Up);
    return info;
}

/* Number of OpenMP threads the oracle will use when asked for nthreads<=0. */
ORACLE_API int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
