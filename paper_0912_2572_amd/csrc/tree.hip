// tree.hip -- tree kernels of the TSQR factorization on gfx950 (Sec. 2.3):
// the structured QR of [R_l; R_r] on the domain triangles, one launch per
// tree level, one workgroup per chain of combines.  The right child's
// triangle is overwritten by the combine's reflector block and its T is
// stored under the right child's index; then the root's R is sign-normalised.
#include "common.h"
#include "factor_common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

// Column steps of one tree combine.  Thread (w, l) of the four waves owns
// column k = 16 w + (l & 15) of the right triangle, rows 16 q .. 16 q + 15
// with q = l >> 4, in c; the left triangle R, which step j changes only in
// row j, is in sm.R (row-major).  The right triangle is upper triangular
// and stays so.  At step j the four threads of column j have put its rows
// in LDS (double-buffered by step parity); every thread reads its quarter
// of x = column j and forms its partial dot with its own column and its
// partial ||x||^2, and the quarters are summed inside the wave (the same
// instructions in every wave, so every thread holds the same scalars):
//     alpha = R[j][j], sig2 = ||x||^2, (beta, tau, s) as in the leaf,
//     k > j:  w = R[j][k] + s d_k,  c_k -= (tau w s) x,  R[j][k] -= tau w,
//     k = j:  R[j][j] = beta; the column keeps x and its scale s_j waits,
//     k < j:  G[k][j] = s_k s d_k (c_k is the unscaled reflector of step k).
// Then the threads of column j + 1 publish its updated rows for the next
// step: one barrier per step.  Row j + 1 of R, final by then, is read
// before that barrier; R[j][j], which every thread reads during step j, is
// written once after the last step.  On exit c holds the reflector block V
// (column k scaled by s_k), sm.R the combined triangle and, if want_t,
// sm.tau and the Gram entries (lower triangle of sm.T).
__device__ __forceinline__ void combine_steps(FactorSmem &sm, double (&c)[16], const int n, const bool want_t) {
    const int t = threadIdx.x, k = 16 * (t >> 6) + (t & 15), q = (t >> 4) & 3;
    // xb[par][64]; its LDS address is past the 16-bit offset field of the
    // DS instructions, so an opaque zero keeps it in one base register with
    // immediate offsets from there
    int zero = 0;
    asm volatile("" : "+v"(zero));
    double *xb = sm.u.P + zero;
    auto publish = [&](int par) {
#pragma unroll
        for (int i = 0; i < 16; ++i) xb[64 * par + 16 * q + i] = c[i];
    };
    if (k == 0) publish(0);
    double alpha = sm.R[0], e = sm.R[k];
    __syncthreads();
    double my_s = 1.0, my_beta = 0.0;
#pragma unroll 1
    for (int j = 0; j < n; ++j) {
        const int par = j & 1;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; i += 2) {
            const dv2 v = *reinterpret_cast<const dv2 *>(xb + 64 * par + 16 * q + i);
            x[i] = v.x;
            x[i + 1] = v.y;
        }
        double p0 = 0.0, p1 = 0.0, s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < 16; i += 2) {
            p0 = fma(x[i], c[i], p0);
            p1 = fma(x[i + 1], c[i + 1], p1);
            s0 = fma(x[i], x[i], s0);
            s1 = fma(x[i + 1], x[i + 1], s1);
        }
        const double d = pair_sum32(pair_sum16(p0 + p1));
        const double sig2 = pair_sum32(pair_sum16(s0 + s1));
        double beta, tau, s;
        householder_scalars(alpha, sig2, beta, tau, s);
        const double wv = fma(s, d, e);
        const bool upd = k > j && k < n;
        const double f = upd ? (tau * wv) * s : 0.0;
        if (q == 0) {
            if (upd) sm.R[j * kLdsStride + k] = e - tau * wv;
            if (want_t && k < j) gram(sm, k, j) = my_s * (s * d);
        }
        if (k == j) {
            my_s = s;
            my_beta = beta;
        }
        if (t == 0) sm.tau[j] = tau;
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = fma(-f, x[i], c[i]);
        if (k == j + 1) publish(par ^ 1);
        if (j + 1 < n) {
            alpha = sm.R[(j + 1) * kLdsStride + j + 1];
            e = sm.R[(j + 1) * kLdsStride + k];
        }
        __syncthreads();
    }
    if (q == 0 && k < n) sm.R[k * kLdsStride + k] = my_beta;
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] *= my_s;
}

// Rows 16 q .. 16 q + 15 of column k (thread layout of combine_steps) of an
// n x n column-major block; zeros outside it.
__device__ __forceinline__ void load_quarter(double (&c)[16], const double *__restrict__ src, int n) {
    const int t = threadIdx.x, k = 16 * (t >> 6) + (t & 15), q = (t >> 4) & 3;
    const double *p = src + (int64_t)(k < n ? k : 0) * n + 16 * q;
    const bool vec = (n % 2) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0;
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
        const int r = 16 * q + i;
        if (vec) {
            const dv2 v = (r < n) ? *reinterpret_cast<const dv2 *>(p + i) : dv2{0.0, 0.0};
            c[i] = v.x;
            c[i + 1] = v.y;
        } else {
            c[i] = (r < n) ? p[i] : 0.0;
            c[i + 1] = (r + 1 < n) ? p[i + 1] : 0.0;
        }
    }
    if (k >= n) {
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = 0.0;
    }
}

__device__ __forceinline__ void store_quarter(const double (&c)[16], double *__restrict__ dst, int n) {
    const int t = threadIdx.x, k = 16 * (t >> 6) + (t & 15), q = (t >> 4) & 3;
    if (k >= n) return;
    double *p = dst + (int64_t)k * n + 16 * q;
    const bool vec = (n % 2) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
        const int r = 16 * q + i;
        if (r < n) {
            if (vec) {
                dv2 v;
                v.x = c[i];
                v.y = c[i + 1];
                *reinterpret_cast<dv2 *>(p + i) = v;
            } else {
                p[i] = c[i];
                if (r + 1 < n) p[i + 1] = c[i + 1];
            }
        }
    }
}

// One chain of combines (step 3): left <- qr([R_left; R_right]) for every
// right = left + q stride (q = 1, 2, ... while q stride < span and right < P),
// in order.  The right triangle is overwritten by the combine's reflector
// block V and, if keep_q, the node's T slot by its Gram entries and tau
// (k_tree_t turns them into T once the whole tree is done, off the chain of
// dependent levels).  The steps read only the upper triangle of sm.R and the
// Gram entries they wrote, so no LDS is cleared.
__device__ __forceinline__ void tree_chain(FactorSmem &sm, double *__restrict__ Rdom,
                                           double *__restrict__ Tnode, const PanelArgs &pa,
                                           int64_t left, int64_t stride, int64_t span, int keep_q) {
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const bool want_t = keep_q != 0;
    double c[16];
    if (stride < span && left + stride < pa.P) load_quarter(c, Rdom + (left + stride) * nn, n);
    {
        // the left triangle, every load in flight before the LDS stores
        double rv[64 * 64 / kFactorThreads];
#pragma unroll
        for (int u = 0; u < 64 * 64 / kFactorThreads; ++u) {
            const int e = threadIdx.x + kFactorThreads * u;
            rv[u] = (e < n * n) ? Rdom[left * nn + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 64 * 64 / kFactorThreads; ++u) {
            const int e = threadIdx.x + kFactorThreads * u;
            const int r = e % n, k = e / n;
            if (e < n * n && r <= k) sm.R[r * kLdsStride + k] = rv[u];
        }
    }
    __syncthreads();
    for (int64_t q = 1; q * stride < span; ++q) {
        const int64_t right = left + q * stride;
        if (right >= pa.P) break;
        if (q > 1) load_quarter(c, Rdom + right * nn, n);
        combine_steps(sm, c, n, want_t);
        // the right triangle becomes the node's reflector block V
        store_quarter(c, Rdom + right * nn, n);
        __syncthreads();
        if (want_t) store_gram(sm, Tnode + right * nn, n);
        __syncthreads();
    }
    store_tri(sm.R, Rdom + left * nn, n);
}

// Every tree node's T: nodes 1 .. P - 1 (each domain but 0 is absorbed as
// the right operand of exactly one combine, whatever the tree's shape).
__global__ __launch_bounds__(kFactorThreads) void k_tree_t(double *__restrict__ Tnode, PanelArgs pa) {
    extern __shared__ double smem_raw[];
    FactorSmem &sm = *reinterpret_cast<FactorSmem *>(smem_raw);
    const int64_t node = 1 + (int64_t)blockIdx.x;
    if (node >= pa.P) return;
    node_t(sm, Tnode + node * (int64_t)pa.n * pa.n, pa.n);
}

__global__ __launch_bounds__(kFactorThreads) void k_tree(double *__restrict__ Rdom, double *__restrict__ Tnode,
                                                         PanelArgs pa, TreeArgs ta, int keep_q) {
    extern __shared__ double smem_raw[];
    FactorSmem &sm = *reinterpret_cast<FactorSmem *>(smem_raw);
    // The levels are the critical path while a solve's leaf passes share the
    // CUs: the chain's waves take the issue slots first.
    __builtin_amdgcn_s_setprio(3);
    const int64_t left = tree_left(ta, blockIdx.x);
    if (left >= pa.P) return;
    tree_chain(sm, Rdom, Tnode, pa, left, ta.stride, ta.span, keep_q);
}

// R_out = D R_root with D = diag(sgn R_jj), sgn(0) = +1; d_out = diag(D).
__global__ void k_sign_normalise(const double *__restrict__ Rroot, int n, double *__restrict__ Rout,
                                 int64_t ldr, int row_off, int col_off, double *__restrict__ dsign) {
    for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < n * n; e += blockDim.x * gridDim.x) {
        const int r = e % n, k = e / n;
        const double dr = (Rroot[r + r * n] < 0.0) ? -1.0 : 1.0;
        Rout[(row_off + r) + (int64_t)(col_off + k) * ldr] = (r <= k) ? dr * Rroot[e] : 0.0;
        if (k == 0) dsign[row_off + r] = dr;
    }
}

size_t factor_smem_bytes() { return sizeof(FactorSmem); }

// ---- batched forms: grid.y walks the matrix list, grid.x the chains of the
// listed matrix (a workgroup past its matrix's count returns).
__global__ __launch_bounds__(kFactorThreads) void k_tree_b(const BMat *__restrict__ mats,
                                                           const int *__restrict__ list, int level) {
    extern __shared__ double smem_raw[];
    FactorSmem &sm = *reinterpret_cast<FactorSmem *>(smem_raw);
    const BMat &M = mats[list[blockIdx.y]];
    if (level >= M.nlev) return;
    const TreeArgs ta = M.lev[level];
    if ((int64_t)blockIdx.x >= ta.chains) return;
    const int64_t left = tree_left(ta, blockIdx.x);
    if (left >= M.pa.P) return;
    tree_chain(sm, M.Rdom, M.Tnode, M.pa, left, ta.stride, ta.span, 1);
}

__global__ __launch_bounds__(kFactorThreads) void k_tree_t_b(const BMat *__restrict__ mats,
                                                             const int *__restrict__ list) {
    extern __shared__ double smem_raw[];
    FactorSmem &sm = *reinterpret_cast<FactorSmem *>(smem_raw);
    const BMat &M = mats[list[blockIdx.y]];
    const int64_t node = 1 + (int64_t)blockIdx.x;
    if (node >= M.pa.P) return;
    node_t(sm, M.Tnode + node * (int64_t)M.pa.n * M.pa.n, M.pa.n);
}

__global__ void k_sign_b(const BMat *__restrict__ mats, const int *__restrict__ list) {
    const BMat &M = mats[list[blockIdx.x]];
    const int n = M.pa.n;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e % n, k = e / n;
        const double dr = (M.Rdom[r + r * n] < 0.0) ? -1.0 : 1.0;
        M.R[e] = (r <= k) ? dr * M.Rdom[e] : 0.0;
        if (k == 0) M.dsign[r] = dr;
    }
}

hipError_t launch_tree_b(const BMat *mats, const int *list, int cnt, int64_t gx, int /*ns*/, int level,
                         hipStream_t st) {
    if (cnt <= 0 || gx <= 0) return hipSuccess;
    const size_t sh = sizeof(FactorSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree_b, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("batch_tree_factor", st);
    hipLaunchKernelGGL(k_tree_b, dim3((unsigned)gx, (unsigned)cnt), dim3(kFactorThreads), sh, st, mats, list,
                       level);
    return hipGetLastError();
}

hipError_t launch_tree_t_b(const BMat *mats, const int *list, int cnt, int64_t maxP, hipStream_t st) {
    if (cnt <= 0 || maxP <= 1) return hipSuccess;
    const size_t sh = sizeof(FactorSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree_t_b, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("batch_tree_t", st);
    hipLaunchKernelGGL(k_tree_t_b, dim3((unsigned)(maxP - 1), (unsigned)cnt), dim3(kFactorThreads), sh, st, mats,
                       list);
    return hipGetLastError();
}

hipError_t launch_sign_b(const BMat *mats, const int *list, int cnt, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    ProfScope ps("batch_sign_normalise", st);
    hipLaunchKernelGGL(k_sign_b, dim3((unsigned)cnt), dim3(256), 0, st, mats, list);
    return hipGetLastError();
}

hipError_t launch_tree_level(double *Rdom, double *Tnode, const PanelArgs &pa, const TreeArgs &ta,
                             int keep_q, hipStream_t st) {
    // one lane per column: n <= 64
    const size_t sh = sizeof(FactorSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("tree_factor", st);
    hipLaunchKernelGGL(k_tree, dim3((unsigned)ta.chains), dim3(kFactorThreads), sh, st, Rdom, Tnode, pa, ta,
                       keep_q);
    return hipGetLastError();
}

hipError_t launch_tree_t(double *Tnode, const PanelArgs &pa, hipStream_t st) {
    if (pa.P <= 1) return hipSuccess;
    const size_t sh = sizeof(FactorSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree_t, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("tree_t", st);
    hipLaunchKernelGGL(k_tree_t, dim3((unsigned)(pa.P - 1)), dim3(kFactorThreads), sh, st, Tnode, pa);
    return hipGetLastError();
}

hipError_t launch_sign_normalise(const double *Rroot, int n, double *Rout, int64_t ldr, int row_off,
                                 int col_off, double *dsign, hipStream_t st) {
    ProfScope ps("sign_normalise", st);
    hipLaunchKernelGGL(k_sign_normalise, dim3(16), dim3(256), 0, st, Rroot, n, Rout, ldr, row_off,
                       col_off, dsign);
    return hipGetLastError();
}

}  // namespace tsqr
