// formq.hip -- the thin Q of a single-panel TSQR (n <= 64) on matrix cores.
//
// Q_1 D = Q_full [D; 0] (Sec. 2.2 uniqueness, sign matrix D).  The tree is
// applied top-down first (Sec. 2.3: the reduction tree is reused for Q):
// the root block is S_0 = D, and a node (l, r) with reflector block
// [I; U] and factor T maps its parent block S_l to
//     S_r = -U T S_l,    S_l <- S_l - T S_l.
// Each domain then expands its n x n block S_i through its chunks, last
// chunk first.  A chunk k >= 1 with reflectors [I; V_k] and factor T_k
// turns the running block X (the domain's top rows) into
//     rows of chunk k = -V_k (T_k X),   X <- X - T_k X,
// and the first chunk (unit lower trapezoidal V_0) gives
//     rows of chunk 0 = [X; 0] - V_0 T_0 (V_0top^T X).
// The chunk products run as FP64 MFMA tiles in the transposed form
// Q^T-tile = Z^T V^T, so that every store writes 16 consecutive rows of a
// column of the column-major Q.
#include "common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

constexpr int LD = 64;     // row stride of the 64 x 64 LDS matrices

struct FormSmem {
    double X[64 * LD];
    double Z[64 * LD];
    double T[64 * LD];
    double W[64 * LD];
};

// Loads an n x n column-major matrix into a zero-padded 64 x 64 row-major
// LDS matrix (optionally as a unit-lower-trapezoidal block: diagonal 1,
// zeros above).  256 threads; each issues its 16 loads before the first
// LDS store, so the block costs one memory round trip.
__device__ __forceinline__ void load_nn(double *dst, const double *__restrict__ src, int64_t lds,
                                        int n, bool unit_lower) {
    constexpr int kPer = 64 * 64 / 256;
    const int tid = local_tid();
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + 256 * u, r = e & 63, c = e >> 6;
        v[u] = (r < n && c < n) ? src[r + (int64_t)c * lds] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + 256 * u, r = e & 63, c = e >> 6;
        double x = v[u];
        if (unit_lower && r < n && c < n) x = (r == c) ? 1.0 : (r > c ? x : 0.0);
        dst[r * LD + c] = x;
    }
}

// The same block in registers (thread's 16 entries, loads in flight) and
// its later store into the LDS matrix.
__device__ __forceinline__ void fetch_nn(double (&v)[16], const double *__restrict__ src, int64_t lds, int n) {
    const int tid = local_tid();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, r = e & 63, c = e >> 6;
        v[u] = (r < n && c < n) ? src[r + (int64_t)c * lds] : 0.0;
    }
}
__device__ __forceinline__ void put_nn(double *dst, const double (&v)[16]) {
    const int tid = local_tid();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, r = e & 63, c = e >> 6;
        dst[r * LD + c] = v[u];
    }
}

__device__ __forceinline__ void store_nn(double *__restrict__ dst, const double *src, int n) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        dst[e] = src[r * LD + c];
    }
}

// Top-down tree level for the thin Q: one workgroup per chain.
__global__ __launch_bounds__(256) void k_tree_down(const double *__restrict__ Rdom,
                                                   const double *__restrict__ Tnode,
                                                   double *__restrict__ S, PanelArgs pa, TreeArgs ta) {
    extern __shared__ double smem_raw[];
    FormSmem &sm = *reinterpret_cast<FormSmem *>(smem_raw);
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const int64_t left = tree_left(ta, blockIdx.x);
    if (left >= pa.P) return;
    int64_t nr = 0;
    for (int64_t q = 1; q * ta.stride < ta.span && left + q * ta.stride < pa.P; ++q) ++nr;
    {
        // S_l and the first node's T and U: all loads in flight at once
        double xv[16], tv[16], uv[16];
        fetch_nn(xv, S + left * nn, n, n);
        if (nr >= 1) {
            fetch_nn(tv, Tnode + (left + nr * ta.stride) * nn, n, n);
            fetch_nn(uv, Rdom + (left + nr * ta.stride) * nn, n, n);
        }
        put_nn(sm.X, xv);
        if (nr >= 1) {
            put_nn(sm.T, tv);
            put_nn(sm.W, uv);
        }
    }
    for (int64_t q = nr; q >= 1; --q) {
        const int64_t right = left + q * ta.stride;
        __syncthreads();
        if (q < nr) {
            load_nn(sm.T, Tnode + right * nn, n, n, false);
            load_nn(sm.W, Rdom + right * nn, n, n, false);   // U (upper triangular)
            __syncthreads();
        }
        lds_gemm64(sm.T, sm.X, sm.Z, LD, true, false, 1.0);       // Z = T S_l
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) sm.X[e] -= sm.Z[e];
        lds_gemm64(sm.W, sm.Z, sm.T, LD, true, false, -1.0);      // S_r = -U Z
        __syncthreads();
        store_nn(S + right * nn, sm.T, n);
    }
    __syncthreads();
    store_nn(S + left * nn, sm.X, n);
}

// The top levels of the top-down tree in one launch: workgroup g takes the
// domain d = g * dstride (a left of a chain at level lstop - 1), starts from
// the root block D and applies the maps of the nodes on its path down to
// level lstop (the left's S_l <- S_l - T S_l for each later right of its
// chain, then S_r = -U (T S_l) on entering a right) -- the products and
// order of k_tree_down, so the blocks are bitwise the same.  The few upper
// nodes are recomputed by each path through them; in exchange the top
// levels cost one launch and occupy only P / dstride CUs.
__global__ __launch_bounds__(256) void k_tree_down_top(const double *__restrict__ Rdom,
                                                       const double *__restrict__ Tnode,
                                                       const double *__restrict__ dsign,
                                                       double *__restrict__ S, PanelArgs pa, TreePath tp,
                                                       int lstop, int64_t dstride) {
    extern __shared__ double smem_raw[];
    FormSmem &sm = *reinterpret_cast<FormSmem *>(smem_raw);
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const int64_t d = (int64_t)blockIdx.x * dstride;
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int r = e / LD, c = e % LD;
        sm.X[e] = (r == c && r < n) ? dsign[r] : 0.0;
    }
    for (int L = tp.nlev - 1; L >= lstop; --L) {
        const int64_t stride = tp.stride[L], span = tp.span[L];
        const int64_t left = d / span * span;
        const int64_t qd = (d - left) / stride;
        int64_t nr = 0;
        for (int64_t q = 1; q * stride < span && left + q * stride < pa.P; ++q) ++nr;
        for (int64_t q = nr; q > qd; --q) {
            __syncthreads();
            load_nn(sm.T, Tnode + (left + q * stride) * nn, n, n, false);
            __syncthreads();
            lds_gemm64(sm.T, sm.X, sm.Z, LD, true, false, 1.0);   // Z = T S_l
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) sm.X[e] -= sm.Z[e];
        }
        if (qd >= 1) {
            const int64_t right = left + qd * stride;
            __syncthreads();
            load_nn(sm.T, Tnode + right * nn, n, n, false);
            load_nn(sm.W, Rdom + right * nn, n, n, false);   // U (upper triangular)
            __syncthreads();
            lds_gemm64(sm.T, sm.X, sm.Z, LD, true, false, 1.0);   // Z = T S_l
            __syncthreads();
            lds_gemm64(sm.W, sm.Z, sm.X, LD, true, false, -1.0);  // S_r = -U Z
        }
    }
    __syncthreads();
    store_nn(S + d * nn, sm.X, n);
}

// S_0 = D (n x n, column-major).
__global__ void k_seed_root(double *S, int n, const double *d) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        S[e] = (r == c) ? d[r] : 0.0;
    }
}

// Q = -V Z (+ [X; 0] on a first chunk) for the rows of one chunk; wave w
// takes the 16-row tiles 4 w .. 4 w + 3 of every 256-row block.  The wave
// keeps its Z operands in registers for the whole chunk and fetches the next
// two tiles' V while the current tile's products run.
__device__ __forceinline__ void chunk_out(const FormSmem &sm, const double *__restrict__ Vc, int64_t ldv,
                                          double *__restrict__ Qc, int64_t ldq, int64_t valid, int n,
                                          bool first) {
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int kbn = (n + 3) >> 2;
    double za[16][4];
#pragma unroll
    for (int kb = 0; kb < 16; ++kb)
#pragma unroll
        for (int CT = 0; CT < 4; ++CT)
            za[kb][CT] = (kb < kbn) ? sm.Z[(4 * kb + l4) * LD + 16 * CT + l16] : 0.0;
    auto load_v = [&](int64_t tile, double (&vb)[16]) {
        const int64_t row = 16 * tile + l16;
        if (first) {
#pragma unroll
            for (int kb = 0; kb < 16; ++kb) {
                const int col = 4 * kb + l4;
                double v = 0.0;
                if (kb < kbn && row < valid && col < n) {
                    v = Vc[row + (int64_t)col * ldv];
                    if (row <= col) v = (row == col) ? 1.0 : 0.0;
                }
                vb[kb] = v;
            }
        } else {
            // no branch around the loads (so the compiler can keep them in
            // flight): a row past the chunk reads its last row (that output
            // row is not stored) and a column past n reads column n - 1 (it
            // meets a zero row of the padded Z)
            const int64_t rr = row < valid ? row : valid - 1;
#pragma unroll
            for (int kb = 0; kb < 16; ++kb) {
                const int col = 4 * kb + l4;
                vb[kb] = Vc[rr + (int64_t)(col < n ? col : n - 1) * ldv];
            }
        }
    };
    // tiles t, t + 1 (+ 13 past a 4-tile group): two tiles in flight while
    // one computes, in three buffers whose roles rotate through a 3-way
    // unrolled loop (no copies of registers whose loads are still in flight)
    auto next_of = [](int64_t t) { return t + ((t % 4 == 3) ? 13 : 1); };
    int64_t tile = 4 * w;
    double ba[16], bb[16], bc[16];
    if (16 * tile < valid) load_v(tile, ba);
    if (16 * next_of(tile) < valid) load_v(next_of(tile), bb);
    auto step = [&](double (&cur)[16], double (&ahead)[16]) {
        const int64_t t2 = next_of(next_of(tile));
        if (16 * t2 < valid) load_v(t2, ahead);
        const int64_t row = 16 * tile + l16;
        d4 acc[4];
#pragma unroll
        for (int CT = 0; CT < 4; ++CT) acc[CT] = d4_zero();
        // all 16 k-steps, with no branch: past n the Z operand is zero and the
        // V operand finite, so those products add exact zeros
#pragma unroll
        for (int kb = 0; kb < 16; ++kb)
#pragma unroll
            for (int CT = 0; CT < 4; ++CT) acc[CT] = mfma_f64(za[kb][CT], cur[kb], acc[CT]);
        if (!first && n == 64 && 16 * tile + 16 <= valid) {
            // a whole tile of a later chunk: no guard around the stores
#pragma unroll
            for (int CT = 0; CT < 4; ++CT)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Qc[row + (int64_t)(16 * CT + 4 * r + l4) * ldq] = -acc[CT][r];
        } else {
#pragma unroll
            for (int CT = 0; CT < 4; ++CT)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = 16 * CT + 4 * r + l4;
                    if (row < valid && col < n) {
                        double val = -acc[CT][r];
                        if (first && row < n) val += sm.X[row * LD + col];
                        Qc[row + (int64_t)col * ldq] = val;
                    }
                }
        }
        tile = next_of(tile);
    };
    while (16 * tile < valid) {
        step(ba, bc);
        if (16 * tile >= valid) break;
        step(bb, ba);
        if (16 * tile >= valid) break;
        step(bc, bb);
    }
}

__global__ __launch_bounds__(256) void k_form_leaf(const double *__restrict__ V, int64_t ldv,
                                                   const double *__restrict__ Tc,
                                                   const double *__restrict__ S, PanelArgs pa,
                                                   double *__restrict__ Q, int64_t ldq) {
    extern __shared__ double smem_raw[];
    FormSmem &sm = *reinterpret_cast<FormSmem *>(smem_raw);
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const int64_t dom = blockIdx.x;
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    load_nn(sm.X, S + dom * nn, n, n, false);
    // T of the chunk processed next, fetched one chunk ahead
    double tn[16];
    fetch_nn(tn, Tc + (dom_chunk0(pa, dom) + nch - 1) * nn, n, n);
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        const int64_t r0 = row0 + ch * pa.chunk;
        const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
        __syncthreads();
        if (ch > 0) {
            put_nn(sm.T, tn);
            fetch_nn(tn, Tc + (dom_chunk0(pa, dom) + ch - 1) * nn, n, n);
            __syncthreads();
            lds_gemm64(sm.T, sm.X, sm.Z, LD, true, false, 1.0);    // Z = T_k X
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) sm.X[e] -= sm.Z[e];
            // chunk_out reads only Z; X is not read for ch > 0
            chunk_out(sm, V + r0, ldv, Q + r0, ldq, valid, n, false);
        } else {
            load_nn(sm.T, V + r0, ldv, n, true);                     // V_0top (unit lower)
            __syncthreads();
            lds_gemm64(sm.T, sm.X, sm.W, LD, true, true, 1.0);     // W = V_0top^T X
            __syncthreads();
            put_nn(sm.T, tn);
            __syncthreads();
            lds_gemm64(sm.T, sm.W, sm.Z, LD, true, false, 1.0);    // Z = T_0 W
            __syncthreads();
            chunk_out(sm, V + r0, ldv, Q + r0, ldq, valid, n, true);
        }
    }
}

static hipError_t set_smem(const void *k) {
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(FormSmem));
}

hipError_t launch_seed_root(double *S, int n, const double *dsign, hipStream_t st) {
    ProfScope ps("seed_root", st);
    hipLaunchKernelGGL(k_seed_root, dim3(1), dim3(256), 0, st, S, n, dsign);
    return hipGetLastError();
}

hipError_t launch_tree_down_top(const double *Rdom, const double *Tnode, const double *dsign, double *S,
                                const PanelArgs &pa, const TreePath &tp, int lstop, int64_t dstride,
                                hipStream_t st) {
    hipError_t e = set_smem((const void *)k_tree_down_top);
    if (e != hipSuccess) return e;
    ProfScope ps("tree_down", st);
    const int64_t groups = (pa.P + dstride - 1) / dstride;
    hipLaunchKernelGGL(k_tree_down_top, dim3((unsigned)groups), dim3(256), sizeof(FormSmem), st, Rdom, Tnode,
                       dsign, S, pa, tp, lstop, dstride);
    return hipGetLastError();
}

hipError_t launch_tree_down(const double *Rdom, const double *Tnode, double *S, const PanelArgs &pa,
                            const TreeArgs &ta, hipStream_t st) {
    hipError_t e = set_smem((const void *)k_tree_down);
    if (e != hipSuccess) return e;
    ProfScope ps("tree_down", st);
    hipLaunchKernelGGL(k_tree_down, dim3((unsigned)ta.chains), dim3(256), sizeof(FormSmem), st, Rdom,
                       Tnode, S, pa, ta);
    return hipGetLastError();
}

hipError_t launch_form_leaf(const double *V, int64_t ldv, const double *Tc, const double *S,
                            const PanelArgs &pa, double *Q, int64_t ldq, hipStream_t st) {
    hipError_t e = set_smem((const void *)k_form_leaf);
    if (e != hipSuccess) return e;
    ProfScope ps("form_leaf", st);
    hipLaunchKernelGGL(k_form_leaf, dim3((unsigned)pa.P), dim3(256), sizeof(FormSmem), st, V, ldv, Tc, S,
                       pa, Q, ldq);
    return hipGetLastError();
}

}  // namespace tsqr
