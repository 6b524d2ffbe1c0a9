// factor.hip -- leaf and tree kernels of the TSQR factorization on gfx950.
//
// Leaf (Sec. 2.3, "the factorization of a domain is the operation performed
// on the leaves"): one 256-thread workgroup per domain.  The domain is
// streamed from HBM in chunks of `rows` rows that live in registers; the
// domain's triangle R lives in LDS.  The first chunk gets a plain Householder
// QR (its top n rows become R); every later chunk C gets the structured QR of
// [R; C] -- the paper's flat tree (Sec. 2.3) applied inside the domain, so A
// is read exactly once.  Each chunk leaves its reflectors V in place of the
// chunk and its compact-WY factor T (Sec. 2.2: H_1...H_n = I - V T V^T).
//
// Tree (Sec. 2.3): the same structured QR of [R_l; R_r] on the domain
// triangles, one launch per tree level, one workgroup per chain of combines.
// The right child's triangle is overwritten by the combine's reflectors and
// its T is stored under the right child's index.
//
// Register layout of a chunk: lane = rg * 8 + cg (cg = column group 0..7,
// rg = row group 0..7 inside the wave, 32 row groups per workgroup).  A
// thread owns rows {i * 32 + rg_wg : i < RPT} and columns {cg + 8 t : t < NS},
// RPT = 64 / NS.  One column step j of Householder QR needs a single
// reduction: with x = column j, the dots d_k = x . c_k for every column k give
// ||x||^2 (k = j), the update coefficients (k > j) and, for k < j, the entries
// v_k . v_j of the Gram matrix that builds T -- so the step has exactly one
// workgroup barrier.
#include <utility>

#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace tsqr {

struct FactorSmem {
    double R[64 * kLdsStride];   // running triangle, row-major
    double T[64 * kLdsStride];   // compact-WY T of the current chunk, row-major
    double red[2][4][64];        // per-wave partial dots, double-buffered
    double redq[2][4][64];       // per-wave row-j values (first chunk only)
    double z[2][64];             // Gram column for T, double-buffered
};

// T[i][jj] = -tau_jj * sum_{q=i}^{jj-1} T[i][q] z_q (Schreiber-Van Loan
// accumulation of the compact-WY factor, Sec. 2.2).  Four threads per row i.
__device__ __forceinline__ void t_column(FactorSmem &sm, int jj, double tau_jj) {
    const int tid = threadIdx.x;
    const int i = tid >> 2, part = tid & 3;
    double acc = 0.0;
    if (i < jj) {
        const double *z = sm.z[jj & 1];
        for (int q = i + part; q < jj; q += 4) acc = fma(sm.T[i * kLdsStride + q], z[q], acc);
    }
    acc = sum_quad(acc);
    if (part == 0 && i < jj) sm.T[i * kLdsStride + jj] = -tau_jj * acc;
    if (tid == 0) sm.T[jj * kLdsStride + jj] = tau_jj;
}

// State carried across the column steps of one chunk.
template <int NS>
struct StepState {
    double tau_prev = 0.0;
    double rnew[NS];     // new R row, written one step late (see below)
    int jprev = -1;
};

// Column steps j = 8 TJ .. 8 TJ + 7 (< n) of chunk_qr.  TJ is a template
// parameter so that the slot index of column j is known at compile time.
template <int NS, int TJ>
__device__ __forceinline__ void qr_steps(double (&c)[rows_per_thread(NS)][NS], const int n,
                                         const bool first, FactorSmem &sm, const bool want_t,
                                         StepState<NS> &ss) {
    constexpr int RPT = rows_per_thread(NS);
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, cg = lane & 7, rgl = lane >> 3;
    const int rg = w * 8 + rgl;
    for (int q = 0; q < 8; ++q) {
        const int j = TJ * 8 + q;
        if (j >= n) return;
        const int par = j & 1;
        // x = column j of this thread's rows (owner lane rg*8 + q)
        double x[RPT];
        const int src = (rgl << 3) | q;
#pragma unroll
        for (int i = 0; i < RPT; ++i) x[i] = __shfl(c[i][TJ], src);
        // first chunk: row j is the pivot row; its values go to the R row
        // (reduced as qv) and it is left out of the dots.
        const bool own_j = first && (rg == (j & 31));
        const int ij = j >> 5;
        double qv[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) qv[t] = 0.0;
        if (own_j) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (i == ij) {
#pragma unroll
                    for (int t = 0; t < NS; ++t) qv[t] = c[i][t];
                    x[i] = 0.0;
                }
        }
        double p[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) s = fma(x[i], c[i][t], s);
            p[t] = s;
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) p[t] = sum_rowgroups(p[t]);
#pragma unroll
        for (int t = 0; t < NS; ++t)
            if (rgl == t) sm.red[par][w][cg + 8 * t] = p[t];
        if (first) {
#pragma unroll
            for (int t = 0; t < NS; ++t) qv[t] = sum_rowgroups(qv[t]);
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (rgl == t) sm.redq[par][w][cg + 8 * t] = qv[t];
        }
        __syncthreads();
        // deferred write of the previous step's R row: every thread has
        // read that row before this barrier.
        if (ss.jprev >= 0 && rg == 0) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const int k = cg + 8 * t;
                if (k >= ss.jprev) sm.R[ss.jprev * kLdsStride + k] = ss.rnew[t];
            }
        }
        double d[NS], e[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 8 * t;
            d[t] = ((sm.red[par][0][k] + sm.red[par][1][k]) + sm.red[par][2][k]) + sm.red[par][3][k];
        }
        const double sig2 =
            ((sm.red[par][0][j] + sm.red[par][1][j]) + sm.red[par][2][j]) + sm.red[par][3][j];
        double alpha;
        if (first) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const int k = cg + 8 * t;
                e[t] = ((sm.redq[par][0][k] + sm.redq[par][1][k]) + sm.redq[par][2][k]) +
                       sm.redq[par][3][k];
            }
            alpha = ((sm.redq[par][0][j] + sm.redq[par][1][j]) + sm.redq[par][2][j]) +
                    sm.redq[par][3][j];
        } else {
#pragma unroll
            for (int t = 0; t < NS; ++t) e[t] = sm.R[j * kLdsStride + cg + 8 * t];
            alpha = sm.R[j * kLdsStride + j];
        }
        double beta, tau, s;
        householder_scalars(alpha, sig2, beta, tau, s);
        if (want_t && j > 0) t_column(sm, j - 1, ss.tau_prev);
        // trailing update (k > j), reflector (k == j), Gram entries (k < j)
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 8 * t;
            if (t < TJ) {
                if (want_t && rg == 0) sm.z[par][k] = (first ? e[t] : 0.0) + s * d[t];
                continue;
            }
            if (k > j) {
                const double wv = e[t] + s * d[t];
                const double f = tau * wv * s;
#pragma unroll
                for (int i = 0; i < RPT; ++i) c[i][t] = fma(-f, x[i], c[i][t]);
                if (own_j) {
#pragma unroll
                    for (int i = 0; i < RPT; ++i)
                        if (i == ij) c[i][t] = 0.0;
                }
                ss.rnew[t] = e[t] - tau * wv;
            } else if (k == j) {
#pragma unroll
                for (int i = 0; i < RPT; ++i) c[i][t] = s * x[i];
                ss.rnew[t] = beta;
            } else {
                if (want_t && rg == 0) sm.z[par][k] = (first ? e[t] : 0.0) + s * d[t];
            }
        }
        ss.tau_prev = tau;
        ss.jprev = j;
    }
}

template <int NS, int... TJ>
__device__ __forceinline__ void qr_all_steps(std::integer_sequence<int, TJ...>,
                                             double (&c)[rows_per_thread(NS)][NS], const int n,
                                             const bool first, FactorSmem &sm, const bool want_t,
                                             StepState<NS> &ss) {
    (qr_steps<NS, TJ>(c, n, first, sm, want_t, ss), ...);
}

// Householder QR of [R; C] (first == false) or of C alone (first == true,
// rows 0..n-1 of C become R).  On exit c holds the reflector tails V (zeros
// on and above the diagonal of a first chunk, whose unit diagonal is
// implicit), sm.R the updated triangle and, if want_t, sm.T the chunk's T.
template <int NS>
__device__ __forceinline__ void chunk_qr(double (&c)[rows_per_thread(NS)][NS], const int n,
                                         const bool first, FactorSmem &sm, const bool want_t) {
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, cg = lane & 7, rgl = lane >> 3;
    const int rg = w * 8 + rgl;
    StepState<NS> ss;
    qr_all_steps<NS>(std::make_integer_sequence<int, NS>{}, c, n, first, sm, want_t, ss);
    __syncthreads();
    if (ss.jprev >= 0 && rg == 0) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 8 * t;
            if (k >= ss.jprev) sm.R[ss.jprev * kLdsStride + k] = ss.rnew[t];
        }
    }
    if (want_t && ss.jprev >= 0) t_column(sm, ss.jprev, ss.tau_prev);
    __syncthreads();
}

// Loads rows [0, valid) x columns [0, n) of a chunk at src (ld) into c.
template <int NS>
__device__ __forceinline__ void load_chunk(double (&c)[rows_per_thread(NS)][NS], const double *__restrict__ src,
                                           int64_t ld, int64_t valid, int n) {
    constexpr int RPT = rows_per_thread(NS);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, cg = lane & 7, rgl = lane >> 3;
    const int rg = w * 8 + rgl;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = (int64_t)i * 32 + rg;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 8 * t;
            c[i][t] = (r < valid && k < n) ? src[r + (int64_t)k * ld] : 0.0;
        }
    }
}

template <int NS>
__device__ __forceinline__ void store_chunk(const double (&c)[rows_per_thread(NS)][NS], double *__restrict__ dst,
                                            int64_t ld, int64_t valid, int n) {
    constexpr int RPT = rows_per_thread(NS);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, cg = lane & 7, rgl = lane >> 3;
    const int rg = w * 8 + rgl;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = (int64_t)i * 32 + rg;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 8 * t;
            if (r < valid && k < n) dst[r + (int64_t)k * ld] = c[i][t];
        }
    }
}

__device__ __forceinline__ void store_tri(const double *lds, double *__restrict__ dst, int n) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e % n, k = e / n;     // column-major n x n
        dst[e] = (r <= k) ? lds[r * kLdsStride + k] : 0.0;
    }
}

__device__ __forceinline__ void zero_lds(double *lds) {
    for (int e = threadIdx.x; e < 64 * kLdsStride; e += blockDim.x) lds[e] = 0.0;
}

template <int NS>
__global__ __launch_bounds__(256) void k_leaf(const double *__restrict__ A, int64_t lda,
                                              double *__restrict__ V, int64_t ldv,
                                              double *__restrict__ Tc, double *__restrict__ Rdom,
                                              PanelArgs pa, int keep_q) {
    extern __shared__ double smem_raw[];
    FactorSmem &sm = *reinterpret_cast<FactorSmem *>(smem_raw);
    constexpr int ROWS = 32 * rows_per_thread(NS);
    const int64_t dom = blockIdx.x;
    const int64_t row0 = dom * pa.mb;
    const int64_t nrows = (dom == pa.P - 1) ? pa.m - row0 : pa.mb;
    const int64_t nch = (nrows + ROWS - 1) / ROWS;
    const int n = pa.n;
    zero_lds(sm.R);
    zero_lds(sm.T);
    __syncthreads();
    double c[rows_per_thread(NS)][NS];
    for (int64_t ch = 0; ch < nch; ++ch) {
        const int64_t r0 = row0 + ch * ROWS;
        const int64_t valid = (nrows - ch * ROWS < ROWS) ? nrows - ch * ROWS : ROWS;
        load_chunk<NS>(c, A + r0, lda, valid, n);
        chunk_qr<NS>(c, n, ch == 0, sm, keep_q != 0);
        if (keep_q) {
            store_chunk<NS>(c, V + r0, ldv, valid, n);
            store_tri(sm.T, Tc + (dom * pa.cpd + ch) * (int64_t)n * n, n);
            __syncthreads();
        }
    }
    store_tri(sm.R, Rdom + dom * (int64_t)n * n, n);
}

// One chain of combines per workgroup: left <- qr([R_left; R_right]) for
// every right of the chain, in order.
template <int NS>
__global__ __launch_bounds__(256) void k_tree(double *__restrict__ Rdom, double *__restrict__ Tnode,
                                              PanelArgs pa, TreeArgs ta, int keep_q) {
    extern __shared__ double smem_raw[];
    FactorSmem &sm = *reinterpret_cast<FactorSmem *>(smem_raw);
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const int64_t left = (int64_t)blockIdx.x * ta.span;
    zero_lds(sm.R);
    zero_lds(sm.T);
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e % n, k = e / n;
        if (r <= k) sm.R[r * kLdsStride + k] = Rdom[left * nn + e];
    }
    __syncthreads();
    double c[rows_per_thread(NS)][NS];
    for (int64_t q = 1; q * ta.stride < ta.span; ++q) {
        const int64_t right = left + q * ta.stride;
        if (right >= pa.P) break;
        load_chunk<NS>(c, Rdom + right * nn, n, n, n);
        chunk_qr<NS>(c, n, false, sm, keep_q != 0);
        // the right triangle becomes the node's reflector block U
        store_chunk<NS>(c, Rdom + right * nn, n, n, n);
        if (keep_q) store_tri(sm.T, Tnode + right * nn, n);
        __syncthreads();
    }
    store_tri(sm.R, Rdom + left * nn, n);
}

// R_out = D R_root with D = diag(sgn R_jj), sgn(0) = +1; d_out = diag(D).
__global__ void k_sign_normalise(const double *__restrict__ Rroot, int n, double *__restrict__ Rout,
                                 int64_t ldr, int row_off, int col_off, int nfull,
                                 double *__restrict__ dsign) {
    for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < n * n; e += blockDim.x * gridDim.x) {
        const int r = e % n, k = e / n;
        const double dr = (Rroot[r + r * n] < 0.0) ? -1.0 : 1.0;
        Rout[(row_off + r) + (int64_t)(col_off + k) * ldr] = (r <= k) ? dr * Rroot[e] : 0.0;
        if (k == 0) dsign[row_off + r] = dr;
    }
    (void)nfull;
}

size_t factor_smem_bytes() { return sizeof(FactorSmem); }

template <int NS>
static hipError_t launch_leaf_ns(const double *A, int64_t lda, double *V, int64_t ldv, double *Tc,
                                 double *Rdom, const PanelArgs &pa, int keep_q, hipStream_t st) {
    const size_t sh = sizeof(FactorSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_leaf<NS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("leaf_factor", st);
    hipLaunchKernelGGL(k_leaf<NS>, dim3((unsigned)pa.P), dim3(256), sh, st, A, lda, V, ldv, Tc, Rdom,
                       pa, keep_q);
    return hipGetLastError();
}

hipError_t launch_leaf(const double *A, int64_t lda, double *V, int64_t ldv, double *Tc, double *Rdom,
                       const PanelArgs &pa, int keep_q, hipStream_t st) {
    switch (pa.ns) {
        case 1: return launch_leaf_ns<1>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, st);
        case 2: return launch_leaf_ns<2>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, st);
        case 4: return launch_leaf_ns<4>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, st);
        default: return launch_leaf_ns<8>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, st);
    }
}

template <int NS>
static hipError_t launch_tree_ns(double *Rdom, double *Tnode, const PanelArgs &pa, const TreeArgs &ta,
                                 int keep_q, hipStream_t st) {
    const size_t sh = sizeof(FactorSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree<NS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("tree_factor", st);
    hipLaunchKernelGGL(k_tree<NS>, dim3((unsigned)ta.chains), dim3(256), sh, st, Rdom, Tnode, pa, ta,
                       keep_q);
    return hipGetLastError();
}

hipError_t launch_tree_level(double *Rdom, double *Tnode, const PanelArgs &pa, const TreeArgs &ta,
                             int keep_q, hipStream_t st) {
    // the tree tile must hold n rows: 32 * rows_per_thread(NS) >= 64 >= n
    switch (pa.ns) {
        case 1: return launch_tree_ns<1>(Rdom, Tnode, pa, ta, keep_q, st);
        case 2: return launch_tree_ns<2>(Rdom, Tnode, pa, ta, keep_q, st);
        case 4: return launch_tree_ns<4>(Rdom, Tnode, pa, ta, keep_q, st);
        default: return launch_tree_ns<8>(Rdom, Tnode, pa, ta, keep_q, st);
    }
}

hipError_t launch_sign_normalise(const double *Rroot, int n, double *Rout, int64_t ldr, int row_off,
                                 int col_off, double *dsign, hipStream_t st) {
    ProfScope ps("sign_normalise", st);
    hipLaunchKernelGGL(k_sign_normalise, dim3(16), dim3(256), 0, st, Rroot, n, Rout, ldr, row_off,
                       col_off, 0, dsign);
    return hipGetLastError();
}

}  // namespace tsqr
