// apply.hip -- applying the TSQR orthogonal factor to a block of columns.
//
// Q is the product of the leaf factors (one per chunk of every domain) and
// the tree factors (one per combine), each in compact-WY form
// I - Y T Y^T (Sec. 2.2).  Q^T B runs the leaves first, chunk by chunk in
// factorization order, then the tree bottom-up; Q B runs the same pieces in
// the reverse order with T in place of T^T (Sec. 2.3: the tree that reduced
// R is reused for Q, Property 1 of Sec. 4).
//
// A chunk k >= 1 of a domain has Y = [I; V_k] on the rows [domain top n rows;
// chunk rows], so with the n-row block Yb (the domain's top rows of B):
//     W = Yb + V_k^T B_k,  W <- T_k^T W (or T_k W),  Yb -= W,  B_k -= V_k W.
// The first chunk of a domain has a plain unit-lower-trapezoidal V_0.
// A tree node (l, r) has Y = [I; U] with U the n x n upper triangle stored
// in the right child's slot, acting on the top n rows of domains l and r.
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace tsqr {

constexpr int KB = 8;          // columns of B per workgroup
constexpr int SB = 64;         // rows per LDS sub-block

struct ApplySmem {
    double Vs[SB * kLdsStride];   // sub-block of V, row-major [row][refl]
    double Ts[64 * kLdsStride];   // T, row-major
    double Bs[SB][KB];
    double Ws[64][KB];
    double Ys[64][KB];
};

// W[i][c] (+)= sum over the chunk's rows of V[r][i] * B[r][c]; then
// B[r][c] -= sum_i V[r][i] W[i][c].  `first` marks a domain's first chunk
// (implicit unit diagonal, zeros above it).  For trans == 0 on a first chunk
// the rows r < n of B are taken from / returned to Ys.
__device__ void chunk_apply(ApplySmem &sm, const double *__restrict__ Vc, int64_t ldv,
                            const double *__restrict__ Tk, const double *__restrict__ Bin,
                            int64_t ldbi, double *__restrict__ Bout, int64_t ldbo, int64_t valid,
                            int n, int kc, bool first, int trans) {
    const int tid = threadIdx.x;
    const int wi = tid & 63, wc = tid >> 6;   // W entries (wi, wc) and (wi, wc + 4)
    // stage T
    for (int e = tid; e < n * n; e += 256) {
        const int r = e % n, q = e / n;
        sm.Ts[r * kLdsStride + q] = Tk[e];
    }
    double acc0 = 0.0, acc1 = 0.0;
    if (!first && wi < n) {
        acc0 = sm.Ys[wi][wc];
        acc1 = sm.Ys[wi][wc + 4];
    }
    for (int64_t r0 = 0; r0 < valid; r0 += SB) {
        const int rows = (int)((valid - r0 < SB) ? valid - r0 : SB);
        __syncthreads();
        for (int e = tid; e < SB * 64; e += 256) {
            const int r = e & (SB - 1), i = e >> 6;
            double v = 0.0;
            if (r < rows && i < n) {
                const int64_t gr = r0 + r;
                v = Vc[gr + (int64_t)i * ldv];
                if (first && gr == i) v = 1.0;
            }
            sm.Vs[r * kLdsStride + i] = v;
        }
        for (int e = tid; e < SB * KB; e += 256) {
            const int r = e & (SB - 1), c = e >> 6;
            double b = 0.0;
            const int64_t gr = r0 + r;
            if (r < rows && c < kc) {
                if (first && !trans && gr < n) b = sm.Ys[gr][c];
                else b = Bin[gr + (int64_t)c * ldbi];
            }
            sm.Bs[r][c] = b;
        }
        __syncthreads();
        if (wi < n) {
            for (int r = 0; r < rows; ++r) {
                const double v = sm.Vs[r * kLdsStride + wi];
                acc0 = fma(v, sm.Bs[r][wc], acc0);
                acc1 = fma(v, sm.Bs[r][wc + 4], acc1);
            }
        }
    }
    __syncthreads();
    if (wi < 64) {
        sm.Ws[wi][wc] = acc0;
        sm.Ws[wi][wc + 4] = acc1;
    }
    __syncthreads();
    // W <- T^T W (trans) or T W
    double t0 = 0.0, t1 = 0.0;
    if (wi < n) {
        if (trans) {
            for (int q = 0; q <= wi; ++q) {
                const double tq = sm.Ts[q * kLdsStride + wi];
                t0 = fma(tq, sm.Ws[q][wc], t0);
                t1 = fma(tq, sm.Ws[q][wc + 4], t1);
            }
        } else {
            for (int q = wi; q < n; ++q) {
                const double tq = sm.Ts[wi * kLdsStride + q];
                t0 = fma(tq, sm.Ws[q][wc], t0);
                t1 = fma(tq, sm.Ws[q][wc + 4], t1);
            }
        }
    }
    __syncthreads();
    if (wi < n) {
        sm.Ws[wi][wc] = t0;
        sm.Ws[wi][wc + 4] = t1;
        if (!first) {
            sm.Ys[wi][wc] -= t0;
            sm.Ys[wi][wc + 4] -= t1;
        }
    }
    // B -= V W, sub-block by sub-block (V restaged)
    for (int64_t r0 = 0; r0 < valid; r0 += SB) {
        const int rows = (int)((valid - r0 < SB) ? valid - r0 : SB);
        __syncthreads();
        for (int e = tid; e < SB * 64; e += 256) {
            const int r = e & (SB - 1), i = e >> 6;
            double v = 0.0;
            if (r < rows && i < n) {
                const int64_t gr = r0 + r;
                v = Vc[gr + (int64_t)i * ldv];
                if (first && gr == i) v = 1.0;
            }
            sm.Vs[r * kLdsStride + i] = v;
        }
        for (int e = tid; e < SB * KB; e += 256) {
            const int r = e & (SB - 1), c = e >> 6;
            double b = 0.0;
            const int64_t gr = r0 + r;
            if (r < rows && c < kc) {
                if (first && !trans && gr < n) b = sm.Ys[gr][c];
                else b = Bin[gr + (int64_t)c * ldbi];
            }
            sm.Bs[r][c] = b;
        }
        __syncthreads();
        for (int e = tid; e < SB * KB; e += 256) {
            const int r = e & (SB - 1), c = e >> 6;
            if (r >= rows || c >= kc) continue;
            double s = sm.Bs[r][c];
            for (int i = 0; i < n; ++i) s = fma(-sm.Vs[r * kLdsStride + i], sm.Ws[i][c], s);
            const int64_t gr = r0 + r;
            if (first && trans && gr < n) sm.Ys[gr][c] = s;   // becomes the domain's Y block
            else if (first && !trans && gr < n) Bout[gr + (int64_t)c * ldbo] = s;
            else Bout[gr + (int64_t)c * ldbo] = s;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_leaf_apply(const double *__restrict__ V, int64_t ldv,
                                                    const double *__restrict__ Tc, PanelArgs pa,
                                                    const double *__restrict__ Bsrc, int64_t ldbs,
                                                    double *__restrict__ B, int64_t ldb, int64_t k,
                                                    int trans) {
    extern __shared__ double smem_raw[];
    ApplySmem &sm = *reinterpret_cast<ApplySmem *>(smem_raw);
    const int64_t dom = blockIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * KB;
    const int kc = (int)((k - c0 < KB) ? k - c0 : KB);
    const int n = pa.n;
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    const int64_t nn = (int64_t)n * n;
    const double *Bs0 = Bsrc + c0 * ldbs;
    double *B0 = B + c0 * ldb;
    const int tid = threadIdx.x;
    if (trans) {
        for (int64_t ch = 0; ch < nch; ++ch) {
            const int64_t r0 = row0 + ch * pa.chunk;
            const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
            chunk_apply(sm, V + r0, ldv, Tc + (dom_chunk0(pa, dom) + ch) * nn, Bs0 + r0, ldbs, B0 + r0, ldb,
                        valid, n, kc, ch == 0, 1);
        }
        for (int e = tid; e < n * KB; e += 256) {
            const int r = e % n, c = e / n;
            if (c < kc) B0[row0 + r + (int64_t)c * ldb] = sm.Ys[r][c];
        }
    } else {
        for (int e = tid; e < 64 * KB; e += 256) {
            const int r = e & 63, c = e >> 6;
            sm.Ys[r][c] = (r < n && c < kc) ? Bs0[row0 + r + (int64_t)c * ldbs] : 0.0;
        }
        __syncthreads();
        for (int64_t ch = nch - 1; ch >= 0; --ch) {
            const int64_t r0 = row0 + ch * pa.chunk;
            const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
            chunk_apply(sm, V + r0, ldv, Tc + (dom_chunk0(pa, dom) + ch) * nn, Bs0 + r0, ldbs, B0 + r0, ldb,
                        valid, n, kc, ch == 0, 0);
        }
    }
}

// Tree level: chain g combines rights into left; Y blocks are the top n rows
// of the domains involved.
// One chain of the tree for the KB-column block cblk of B: the chain's
// nodes (left, right) in order (Q^T) or in reverse order (Q).
__device__ __forceinline__ void tree_apply_chain(ApplySmem &sm, const double *__restrict__ Rdom,
                                                 const double *__restrict__ Tnode, const PanelArgs &pa,
                                                 int64_t left, int64_t stride, int64_t span,
                                                 double *__restrict__ B, int64_t ldb, int64_t k, int trans,
                                                 int64_t cblk) {
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const int64_t c0 = cblk * KB;
    const int kc = (int)((k - c0 < KB) ? k - c0 : KB);
    double *B0 = B + c0 * ldb;
    const int tid = threadIdx.x;
    const int wi = tid & 63, wc = tid >> 6;
    int64_t nr = 0;
    for (int64_t q = 1; q * stride < span && left + q * stride < pa.P; ++q) ++nr;
    for (int e = tid; e < 64 * KB; e += 256) {
        const int r = e & 63, c = e >> 6;
        sm.Ys[r][c] = (r < n && c < kc) ? B0[dom_row0(pa, left) + r + (int64_t)c * ldb] : 0.0;
    }
    for (int64_t qq = 0; qq < nr; ++qq) {
        const int64_t q = trans ? qq + 1 : nr - qq;
        const int64_t right = left + q * stride;
        const double *U = Rdom + right * nn;
        const double *T = Tnode + right * nn;
        double *Yr = B0 + dom_row0(pa, right);
        // the node's U and T: every load in flight before the LDS stores
        double uv[16], tv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            uv[u] = (e < n * n) ? U[e] : 0.0;
            tv[u] = (e < n * n) ? T[e] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            if (e < n * n) {
                const int r = e % n, c = e / n;
                sm.Vs[r * kLdsStride + c] = uv[u];
                sm.Ts[r * kLdsStride + c] = tv[u];
            }
        }
        for (int e = tid; e < 64 * KB; e += 256) {
            const int r = e & 63, c = e >> 6;
            sm.Bs[r][c] = (r < n && c < kc) ? Yr[r + (int64_t)c * ldb] : 0.0;
        }
        __syncthreads();
        double a0 = 0.0, a1 = 0.0;
        if (wi < n) {
            a0 = sm.Ys[wi][wc];
            a1 = sm.Ys[wi][wc + 4];
            for (int r = 0; r <= wi; ++r) {
                const double u = sm.Vs[r * kLdsStride + wi];
                a0 = fma(u, sm.Bs[r][wc], a0);
                a1 = fma(u, sm.Bs[r][wc + 4], a1);
            }
        }
        sm.Ws[wi][wc] = a0;
        sm.Ws[wi][wc + 4] = a1;
        __syncthreads();
        double t0 = 0.0, t1 = 0.0;
        if (wi < n) {
            if (trans) {
                for (int q2 = 0; q2 <= wi; ++q2) {
                    const double tq = sm.Ts[q2 * kLdsStride + wi];
                    t0 = fma(tq, sm.Ws[q2][wc], t0);
                    t1 = fma(tq, sm.Ws[q2][wc + 4], t1);
                }
            } else {
                for (int q2 = wi; q2 < n; ++q2) {
                    const double tq = sm.Ts[wi * kLdsStride + q2];
                    t0 = fma(tq, sm.Ws[q2][wc], t0);
                    t1 = fma(tq, sm.Ws[q2][wc + 4], t1);
                }
            }
        }
        __syncthreads();
        if (wi < n) {
            sm.Ws[wi][wc] = t0;
            sm.Ws[wi][wc + 4] = t1;
            sm.Ys[wi][wc] -= t0;
            sm.Ys[wi][wc + 4] -= t1;
        }
        __syncthreads();
        for (int e = tid; e < 64 * KB; e += 256) {
            const int r = e & 63, c = e >> 6;
            if (r >= n || c >= kc) continue;
            double s = sm.Bs[r][c];
            for (int i = r; i < n; ++i) s = fma(-sm.Vs[r * kLdsStride + i], sm.Ws[i][c], s);
            Yr[r + (int64_t)c * ldb] = s;
        }
    }
    __syncthreads();
    for (int e = tid; e < 64 * KB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < n && c < kc) B0[dom_row0(pa, left) + r + (int64_t)c * ldb] = sm.Ys[r][c];
    }
}

__global__ __launch_bounds__(256) void k_tree_apply(const double *__restrict__ Rdom,
                                                    const double *__restrict__ Tnode, PanelArgs pa,
                                                    TreeArgs ta, double *__restrict__ B, int64_t ldb,
                                                    int64_t k, int trans) {
    extern __shared__ double smem_raw[];
    ApplySmem &sm = *reinterpret_cast<ApplySmem *>(smem_raw);
    // A latency-bound chain that may share CUs with a thin Q's top-down tree:
    // its waves take the issue slots first.
    __builtin_amdgcn_s_setprio(3);
    const int64_t left = tree_left(ta, blockIdx.x);
    if (left >= pa.P) return;
    tree_apply_chain(sm, Rdom, Tnode, pa, left, ta.stride, ta.span, B, ldb, k,
                     trans, blockIdx.y);
}

// Batched: level `step` from the bottom (Q^T) or from the top (Q) of each
// listed matrix's own tree, on its vector F.
__global__ __launch_bounds__(256) void k_tree_apply_b(const BMat *__restrict__ mats,
                                                      const int *__restrict__ list, int trans, int step,
                                                      int sweep) {
    extern __shared__ double smem_raw[];
    ApplySmem &sm = *reinterpret_cast<ApplySmem *>(smem_raw);
    const BMat &M = mats[list[blockIdx.y]];
    if (step >= M.nlev) return;
    if (sweep > 0 && M.status[1]) return;
    const TreeArgs ta = M.lev[trans ? step : M.nlev - 1 - step];
    if ((int64_t)blockIdx.x >= ta.chains) return;
    const int64_t left = tree_left(ta, blockIdx.x);
    if (left >= M.pa.P) return;
    tree_apply_chain(sm, M.Rdom, M.Tnode, M.pa, left, ta.stride, ta.span, M.F,
                     M.pa.m, 1, trans, 0);
}

__global__ void k_scale_b(const BMat *__restrict__ mats, const int *__restrict__ list, int sweep) {
    const BMat &M = mats[list[blockIdx.x]];
    if (sweep > 0 && M.status[1]) return;
    for (int r = threadIdx.x; r < M.pa.n; r += blockDim.x) M.F[r] *= M.dsign[r];
}

__global__ void k_scale_rows(double *B, int64_t ldb, int n, int64_t k, const double *d) {
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < (int64_t)n * k;
         e += (int64_t)blockDim.x * gridDim.x) {
        const int r = (int)(e % n);
        const int64_t c = e / n;
        B[r + c * ldb] *= d[r];
    }
}

hipError_t launch_leaf_apply(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                             const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                             int trans, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const size_t sh = sizeof(ApplySmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_leaf_apply,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)pa.P, (unsigned)((k + KB - 1) / KB));
    ProfScope ps(trans ? "leaf_apply_qt" : "leaf_apply_q", st);
    hipLaunchKernelGGL(k_leaf_apply, grid, dim3(256), sh, st, V, ldv, Tc, pa, Bsrc, ldbs, B, ldb, k,
                       trans);
    return hipGetLastError();
}

hipError_t launch_tree_apply(const double *Rdom, const double *Tnode, const PanelArgs &pa,
                             const TreeArgs &ta, double *B, int64_t ldb, int64_t k, int trans,
                             hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const size_t sh = sizeof(ApplySmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree_apply,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)ta.chains, (unsigned)((k + KB - 1) / KB));
    ProfScope ps(trans ? "tree_apply_qt" : "tree_apply_q", st);
    hipLaunchKernelGGL(k_tree_apply, grid, dim3(256), sh, st, Rdom, Tnode, pa, ta, B, ldb, k, trans);
    return hipGetLastError();
}

hipError_t launch_scale_rows(double *B, int64_t ldb, int n, int64_t k, const double *d, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    ProfScope ps("scale_rows", st);
    hipLaunchKernelGGL(k_scale_rows, dim3(8), dim3(256), 0, st, B, ldb, n, k, d);
    return hipGetLastError();
}


hipError_t launch_tree_apply_b(const BMat *mats, const int *list, int cnt, int64_t gx, int trans, int step,
                               int sweep, hipStream_t st) {
    if (cnt <= 0 || gx <= 0) return hipSuccess;
    const size_t sh = sizeof(ApplySmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree_apply_b,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps(trans ? "batch_tree_apply_qt" : "batch_tree_apply_q", st);
    hipLaunchKernelGGL(k_tree_apply_b, dim3((unsigned)gx, (unsigned)cnt), dim3(256), sh, st, mats, list,
                       trans, step, sweep);
    return hipGetLastError();
}

hipError_t launch_scale_b(const BMat *mats, const int *list, int cnt, int sweep, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    ProfScope ps("batch_scale_rows", st);
    hipLaunchKernelGGL(k_scale_b, dim3((unsigned)cnt), dim3(64), 0, st, mats, list, sweep);
    return hipGetLastError();
}

}  // namespace tsqr
