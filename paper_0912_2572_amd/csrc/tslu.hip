// tslu.hip -- LU of a tall-skinny matrix with tournament pivoting (TSLU).
//
// The paper's conclusion carries TSQR's reduction tree over to LU (CALU's
// panel factorization).  What travels up the tree is a set of b candidate
// pivot rows instead of a triangle: a node stacks original rows of A (its
// children's candidates), runs Gaussian elimination with partial pivoting
// on the stack and keeps the b rows chosen as pivots.
//
//   k_tslu_leaf   one workgroup per domain: the domain's rows in stages of
//                 one 256-row stack each (its first 256 rows, then its b
//                 candidates on the next 256 - b rows), the flat tree of
//                 the TSQR leaf's chunks;
//   k_tslu_tree   one workgroup per chain of a tree level (the TSQR tree's
//                 shapes): the left's candidates stacked on each right's;
//   k_tslu_u      U and the unit lower L11 of A[ipiv, :] without pivoting;
//   k_tslu_l      l_i = a_i U^{-1} for every row (one row per thread);
//   k_tslu_scatter  rows ipiv[k] of L <- row k of L11.
//
// Stack layout (256 threads): thread t holds the 16 stack rows 16 (t & 15)
// .. +15 of the four columns 4 (t >> 4) .. +3, so the 16 lanes holding a
// column sit in one 16-lane segment of one wave: the pivot search is a
// 16-lane shuffle reduction, the pivot row's entries come from a lane of the
// thread's own segment, and only the multipliers of the step go through LDS
// (double-buffered: one barrier per elimination step).
#include "kernels.h"
#include "prof.h"

namespace tsqr {

namespace {

constexpr int kStack = 256;

struct TsluSmem {
    double l[2][kStack];     // multipliers of the step (by step parity)
    int32_t gidx[kStack];    // row of A at each stack position
    int32_t sel[64];         // stack positions of the pivots, in order
    int32_t piv[2];          // pivot position of the step (by step parity)
};

typedef double Rows16[16];   // the 16 stack rows one thread holds of one column

// The pivot search and the multipliers of column j (this lane's column jc of
// four) in the 16 lanes holding it; the column index is a template argument
// so that every register access is static.
template <int JC>
__device__ __forceinline__ void pivot_column(TsluSmem &sm, const Rows16 (&a)[4], uint32_t act, int j, int par) {
    const int rb = threadIdx.x & 15;
    double best = -1.0, bv = 0.0;
    int bp = 1 << 30;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        double key = fabs(a[JC][i]);
        if (key != key) key = -0.5;
        if (((act >> i) & 1u) && key > best) {
            best = key;
            bp = 16 * rb + i;
            bv = a[JC][i];
        }
    }
#pragma unroll
    for (int s = 1; s < 16; s <<= 1) {
        const double ob = __shfl_xor(best, s, 16);
        const int op = __shfl_xor(bp, s, 16);
        const double ov = __shfl_xor(bv, s, 16);
        if (ob > best || (ob == best && op < bp)) {
            best = ob;
            bp = op;
            bv = ov;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = 16 * rb + i;
        const bool live = ((act >> i) & 1u) && q != bp && bv != 0.0;
        sm.l[par][q] = live ? a[JC][i] / bv : 0.0;
    }
    if (rb == 0) {
        sm.piv[par] = bp;
        sm.sel[j] = bp;
    }
}

// u[c] = a[c][K]: one case of a branch on the wave-uniform row index.
template <int K>
__device__ __forceinline__ void take_row(const Rows16 (&a)[4], double (&u)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = a[c][K];
}

// Loads the stack: position q holds row gidx[q] of A for q < rows (columns
// past b and positions past rows are zero).  act: this thread's live rows.
__device__ __forceinline__ void load_stack(const TsluSmem &sm, const double *__restrict__ A, int64_t lda,
                                           int rows, int b, Rows16 (&a)[4], uint32_t &act) {
    const int t = threadIdx.x, cg = t >> 4, rb = t & 15;
    act = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = 16 * rb + i;
        const bool live = q < rows;
        if (live) act |= 1u << i;
        const int64_t g = live ? sm.gidx[q] : 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = 4 * cg + c;
            const double v = A[g + (int64_t)(col < b ? col : 0) * lda];
            a[c][i] = (live && col < b) ? v : 0.0;
        }
    }
}

// min(b, rows) steps of partial-pivoting elimination on the stack; the
// pivot positions go to sm.sel.  Ties go to the lower stack position; a
// NaN ranks below every number (a column of NaNs takes its first live row);
// a zero pivot eliminates nothing.  Entries of columns <= j keep being
// updated after their step (never read again), so every column takes the
// same update and no lane branches on its column.
__device__ __forceinline__ void gepp_steps(TsluSmem &sm, Rows16 (&a)[4], uint32_t act, int rows, int b) {
    const int t = threadIdx.x, cg = t >> 4, rb = t & 15;
    const int kb = b < rows ? b : rows;
    for (int j = 0; j < kb; ++j) {
        const int par = j & 1;
        if (cg == (j >> 2)) {
            switch (j & 3) {
                case 0: pivot_column<0>(sm, a, act, j, par); break;
                case 1: pivot_column<1>(sm, a, act, j, par); break;
                case 2: pivot_column<2>(sm, a, act, j, par); break;
                default: pivot_column<3>(sm, a, act, j, par); break;
            }
        }
        __syncthreads();
        const int p = __builtin_amdgcn_readfirstlane(sm.piv[par]);
        const int ip = p & 15, src = p >> 4;
        double u[4];
        switch (ip) {
            case 0: take_row<0>(a, u); break;
            case 1: take_row<1>(a, u); break;
            case 2: take_row<2>(a, u); break;
            case 3: take_row<3>(a, u); break;
            case 4: take_row<4>(a, u); break;
            case 5: take_row<5>(a, u); break;
            case 6: take_row<6>(a, u); break;
            case 7: take_row<7>(a, u); break;
            case 8: take_row<8>(a, u); break;
            case 9: take_row<9>(a, u); break;
            case 10: take_row<10>(a, u); break;
            case 11: take_row<11>(a, u); break;
            case 12: take_row<12>(a, u); break;
            case 13: take_row<13>(a, u); break;
            case 14: take_row<14>(a, u); break;
            default: take_row<15>(a, u); break;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) u[c] = __shfl(u[c], src, 16);
        if (src == rb) act &= ~(1u << ip);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double li = sm.l[par][16 * rb + i];
#pragma unroll
            for (int c = 0; c < 4; ++c) a[c][i] = fma(-li, u[c], a[c][i]);
        }
    }
}

// After gepp_steps: gidx[0 .. kb-1] <- the chosen rows in pivot order.
__device__ __forceinline__ int keep_selection(TsluSmem &sm, int rows, int b) {
    const int kb = b < rows ? b : rows;
    __syncthreads();
    const int t = threadIdx.x;
    const int32_t g = (t < kb) ? sm.gidx[sm.sel[t]] : 0;
    __syncthreads();
    if (t < kb) sm.gidx[t] = g;
    return kb;
}

}  // namespace

__global__ __launch_bounds__(256) void k_tslu_leaf(const double *__restrict__ A, int64_t lda, PanelArgs pa,
                                                   int b, int32_t *__restrict__ cand) {
    __shared__ TsluSmem sm;
    const int64_t dom = blockIdx.x;
    const int64_t row0 = dom_row0(pa, dom), end = row0 + dom_rows(pa, dom);
    const int t = threadIdx.x;
    double a[4][16];
    uint32_t act;
    int64_t pos = row0;
    int nc = 0;
    while (pos < end) {
        const int room = kStack - (nc ? b : 0);
        const int take = (int)((end - pos < room) ? end - pos : room);
        if (t >= nc && t < nc + take) sm.gidx[t] = (int32_t)(pos + (t - nc));
        __syncthreads();
        const int rows = nc + take;
        load_stack(sm, A, lda, rows, b, a, act);
        gepp_steps(sm, a, act, rows, b);
        nc = keep_selection(sm, rows, b);
        pos += take;
        __syncthreads();
    }
    if (t < b) cand[dom * b + t] = sm.gidx[t];
}

__global__ __launch_bounds__(256) void k_tslu_tree(const double *__restrict__ A, int64_t lda, PanelArgs pa,
                                                   TreeArgs ta, int b, int32_t *__restrict__ cand) {
    __shared__ TsluSmem sm;
    const int64_t g = blockIdx.x;
    const int64_t left = (g / ta.width) * ta.span + g % ta.width;
    if (left >= pa.P) return;
    const int t = threadIdx.x;
    double a[4][16];
    uint32_t act;
    for (int64_t q = 1; q * ta.stride < ta.span && left + q * ta.stride < pa.P; ++q) {
        const int64_t right = left + q * ta.stride;
        if (t < b) {
            sm.gidx[t] = cand[left * b + t];
            sm.gidx[b + t] = cand[right * b + t];
        }
        __syncthreads();
        load_stack(sm, A, lda, 2 * b, b, a, act);
        gepp_steps(sm, a, act, 2 * b, b);
        keep_selection(sm, 2 * b, b);
        if (t < b) cand[left * b + t] = sm.gidx[t];
        __syncthreads();
    }
}

// U and the unit lower L11 of A[ipiv, :] by elimination without pivoting:
// thread i owns row i; row j is final after step j - 1.  info: the first
// zero U_jj (1-based), else 0.
__global__ __launch_bounds__(64) void k_tslu_u(const double *__restrict__ A, int64_t lda, int b,
                                               const int32_t *__restrict__ cand, int64_t *__restrict__ ipiv,
                                               double *__restrict__ U, int64_t ldu, double *__restrict__ L11,
                                               int32_t *__restrict__ dinfo) {
    __shared__ double M[64][65];
    const int i = threadIdx.x;
    const int32_t gi = (i < b) ? cand[i] : 0;
    if (i < b) ipiv[i] = gi;
    for (int k = 0; k < b; ++k) M[i][k] = (i < b) ? A[gi + (int64_t)k * lda] : 0.0;
    __syncthreads();
    int info = 0;
    for (int j = 0; j < b; ++j) {
        const double piv = M[j][j];
        if (piv == 0.0) {
            if (!info) info = j + 1;
        } else if (i > j && i < b) {
            const double l = M[i][j] / piv;
            M[i][j] = l;
            for (int k = j + 1; k < b; ++k) M[i][k] = fma(-l, M[j][k], M[i][k]);
        }
        __syncthreads();
    }
    if (i < b) {
        for (int k = 0; k < b; ++k) {
            U[i + (int64_t)k * ldu] = (i <= k) ? M[i][k] : 0.0;
            L11[i + (int64_t)k * 64] = (k < i) ? M[i][k] : (k == i ? 1.0 : 0.0);
        }
    }
    if (i == 0 && dinfo) *dinfo = info;
}

// l_i = a_i U^{-1} (l U = a_i, column by column, l_k = 0 where U_kk = 0)
// for rows i of [0, m); U in LDS, read by every lane at the same address.
__global__ __launch_bounds__(256) void k_tslu_l(const double *__restrict__ A, int64_t lda, int64_t m, int b,
                                                const double *__restrict__ U, int64_t ldu, double *__restrict__ L,
                                                int64_t ldl) {
    __shared__ double Us[64 * 64];
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        Us[e] = (r < b && c < b) ? U[r + (int64_t)c * ldu] : 0.0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double l[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) l[k] = (k < b) ? A[i + (int64_t)k * lda] : 0.0;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        if (k < b) {
            double s = l[k];
#pragma unroll
            for (int j = 0; j < k; ++j) s = fma(-l[j], Us[j + 64 * k], s);
            const double d = Us[k + 64 * k];
            l[k] = (d == 0.0) ? 0.0 : s / d;
        }
    }
#pragma unroll
    for (int k = 0; k < 64; ++k)
        if (k < b) L[i + (int64_t)k * ldl] = l[k];
}

__global__ void k_tslu_scatter(const int64_t *__restrict__ ipiv, int b, const double *__restrict__ L11,
                               double *__restrict__ L, int64_t ldl) {
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int r = e % b, c = e / b;
        L[ipiv[r] + (int64_t)c * ldl] = L11[r + 64 * c];
    }
}

hipError_t launch_tslu(const double *A, int64_t lda, const PanelArgs &pa, const std::vector<TreeArgs> &levels,
                       int b, int32_t *cand, double *L11, double *L, int64_t ldl, double *U, int64_t ldu,
                       int64_t *ipiv, int32_t *dinfo, hipStream_t st) {
    {
        ProfScope ps("tslu_leaf", st);
        hipLaunchKernelGGL(k_tslu_leaf, dim3((unsigned)pa.P), dim3(256), 0, st, A, lda, pa, b, cand);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (const TreeArgs &ta : levels) {
        ProfScope ps("tslu_tree", st);
        hipLaunchKernelGGL(k_tslu_tree, dim3((unsigned)ta.chains), dim3(256), 0, st, A, lda, pa, ta, b, cand);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        ProfScope ps("tslu_u", st);
        hipLaunchKernelGGL(k_tslu_u, dim3(1), dim3(64), 0, st, A, lda, b, cand, ipiv, U, ldu, L11, dinfo);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        ProfScope ps("tslu_l", st);
        const unsigned blocks = (unsigned)((pa.m + 255) / 256);
        hipLaunchKernelGGL(k_tslu_l, dim3(blocks), dim3(256), 0, st, A, lda, pa.m, b, U, ldu, L, ldl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps("tslu_scatter", st);
    hipLaunchKernelGGL(k_tslu_scatter, dim3(1), dim3(256), 0, st, ipiv, b, L11, L, ldl);
    return hipGetLastError();
}

}  // namespace tsqr
