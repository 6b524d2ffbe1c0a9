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
//                 shapes): the left's candidates stacked on each right's,
//                 one thread per stack row (two waves);
//   k_tslu_u      U and the unit lower L11 of A[ipiv, :] without pivoting;
//   k_tslu_l      l_i = a_i U^{-1} for every row (one row per thread);
//   k_tslu_scatter  rows ipiv[k] of L <- row k of L11.
//
// Stack layout (256 threads): thread t holds the stack positions 16 i +
// (t & 15), i = 0..15, of the four columns 4 (t >> 4) .. +3, so the 16 lanes
// holding a column form one 16-lane row of one wave: the pivot search is a
// DPP reduction in that row, the pivot row's entries come from a lane of the
// thread's own row by DPP broadcast, and only the multipliers of the step
// go through LDS (double-buffered: one barrier per elimination step).
#include "common.h"
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

// Lane l of a 16-lane row <- lane N of that row (DPP row_newbcast).
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
    return dpp_f64<0x150 + N>(v);
}

// (value, position) pairs: the larger value wins, equal values go to the
// lower position.
__device__ __forceinline__ void argmax_take(double &best, int &bp, double &bv, double ob, int op, double ov) {
    if (ob > best || (ob == best && op < bp)) {
        best = ob;
        bp = op;
        bv = ov;
    }
}

template <int CTRL>
__device__ __forceinline__ void argmax_step(double &best, int &bp, double &bv) {
    argmax_take(best, bp, bv, dpp_f64<CTRL>(best), __builtin_amdgcn_update_dpp(0, bp, CTRL, 0xf, 0xf, false),
                dpp_f64<CTRL>(bv));
}

// Loads the stack: position q = 16 i + r (r = lane in its 16-lane row, i =
// slot) holds row gidx[q] of A for q < rows, so the 16 lanes of a row read
// 16 consecutive positions of a column per load; columns past b and
// positions past rows are zero.  act: bit i set when slot i is live.  Every
// load is issued before any is used (addresses clamped into A).
__device__ __forceinline__ void load_stack(const TsluSmem &sm, const double *__restrict__ A, int64_t lda,
                                           int rows, int b, Rows16 (&a)[4], uint32_t &act) {
    const int t = threadIdx.x, cg = t >> 4, r = t & 15;
    int64_t g[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = 16 * i + r;
        g[i] = q < rows ? sm.gidx[q] : 0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t co = (int64_t)(4 * cg + c < b ? 4 * cg + c : 0) * lda;
#pragma unroll
        for (int i = 0; i < 16; ++i) a[c][i] = A[g[i] + co];
    }
    act = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const bool live = 16 * i + r < rows;
        if (live) act |= 1u << i;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (!live || 4 * cg + c >= b) a[c][i] = 0.0;
    }
}

// The pivot search and the multipliers of column j (column JC of this
// lane's four) in the 16 lanes holding it; the column index is a template
// argument so that every register access is static.
template <int JC>
__device__ __forceinline__ void pivot_column(TsluSmem &sm, const Rows16 (&a)[4], uint32_t act, int j, int par) {
    const int r = threadIdx.x & 15;
    double best = -1.0, bv = 0.0;
    int bp = 1 << 30;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        double key = fabs(a[JC][i]);
        if (key != key) key = -0.5;
        if (((act >> i) & 1u) && key > best) {
            best = key;
            bp = 16 * i + r;
            bv = a[JC][i];
        }
    }
    argmax_step<kDppXor1>(best, bp, bv);
    argmax_step<kDppXor2>(best, bp, bv);
    argmax_step<0x124>(best, bp, bv);   // row_ror:4: the next quad's winner
    argmax_step<kDppRowRor8>(best, bp, bv);
    // the multipliers only steer the selection (U and L are computed from
    // the chosen rows afterwards): one reciprocal instead of 16 divisions
    const double rv = (bv != 0.0) ? 1.0 / bv : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = 16 * i + r;
        const bool live = ((act >> i) & 1u) && q != bp;
        sm.l[par][q] = live ? a[JC][i] * rv : 0.0;
    }
    if (r == 0) {
        sm.piv[par] = bp;
        sm.sel[j] = bp;
    }
}

// u[c] = a[c][K]: one case of a branch on the wave-uniform slot index.
template <int K>
__device__ __forceinline__ void take_slot(const Rows16 (&a)[4], double (&u)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = a[c][K];
}

template <int N>
__device__ __forceinline__ void bcast_from(double (&u)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = row_bcast<N>(u[c]);
}

// min(b, rows) steps of partial-pivoting elimination on the stack; the
// pivot positions go to sm.sel.  Ties go to the lower stack position; a
// NaN ranks below every number (a column of NaNs takes its first live row);
// a zero pivot eliminates nothing.  Entries of columns <= j keep being
// updated after their step (never read again), so every column takes the
// same update and no lane branches on its column.  The pivot row's entries
// come from the lane of the thread's own 16-lane row that holds it: a
// branch on the (wave-uniform) slot picks the register, a DPP broadcast
// moves it.
__device__ __forceinline__ void gepp_steps(TsluSmem &sm, Rows16 (&a)[4], uint32_t act, int rows, int b) {
    const int t = threadIdx.x, cg = t >> 4, r = t & 15;
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
        const int slot = p >> 4, src = p & 15;
        double u[4];
        switch (slot) {
            case 0: take_slot<0>(a, u); break;
            case 1: take_slot<1>(a, u); break;
            case 2: take_slot<2>(a, u); break;
            case 3: take_slot<3>(a, u); break;
            case 4: take_slot<4>(a, u); break;
            case 5: take_slot<5>(a, u); break;
            case 6: take_slot<6>(a, u); break;
            case 7: take_slot<7>(a, u); break;
            case 8: take_slot<8>(a, u); break;
            case 9: take_slot<9>(a, u); break;
            case 10: take_slot<10>(a, u); break;
            case 11: take_slot<11>(a, u); break;
            case 12: take_slot<12>(a, u); break;
            case 13: take_slot<13>(a, u); break;
            case 14: take_slot<14>(a, u); break;
            default: take_slot<15>(a, u); break;
        }
        switch (src) {
            case 0: bcast_from<0>(u); break;
            case 1: bcast_from<1>(u); break;
            case 2: bcast_from<2>(u); break;
            case 3: bcast_from<3>(u); break;
            case 4: bcast_from<4>(u); break;
            case 5: bcast_from<5>(u); break;
            case 6: bcast_from<6>(u); break;
            case 7: bcast_from<7>(u); break;
            case 8: bcast_from<8>(u); break;
            case 9: bcast_from<9>(u); break;
            case 10: bcast_from<10>(u); break;
            case 11: bcast_from<11>(u); break;
            case 12: bcast_from<12>(u); break;
            case 13: bcast_from<13>(u); break;
            case 14: bcast_from<14>(u); break;
            default: bcast_from<15>(u); break;
        }
        if (src == r) act &= ~(1u << slot);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double li = sm.l[par][16 * i + r];
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

// The tree's stacks hold two candidate sets (2b <= 128 rows): one thread
// per stack row, two waves, the row's 64 entries in registers.  Step J:
//   each wave's argmax of |a_iJ| over its live rows (a NaN ranks below
//   every number, ties go to the lower position: the pivot_column rules)
//   by DPP inside each 16-lane row and lane reads across the four rows; the
//   wave's winner puts its row past J in LDS (one buffer per wave, double-
//   buffered by step parity) with its key; one barrier; every thread takes
//   the better of the two waves' winners, reads that row in one batch and
//   updates its entries past J with l = a_iJ / a_pJ (one reciprocal, as in
//   pivot_column: the multipliers only steer the selection).
struct TreeSelSmem {
    double prow[2][2][64];   // [wave][parity][column]
    double key[2][2];        // [wave][parity]
    double val[2][2];
    int32_t pos[2][2];
    int32_t gidx[128];
    int32_t sel[64];
};

template <int J>
struct TreeSelStep {
    __device__ __forceinline__ static void run(TreeSelSmem &sm, double (&m)[64], bool &live, int b) {
        if (J < b) {
            const int t = threadIdx.x, w = t >> 6, lane = t & 63;
            constexpr int par = J & 1;
            double best = -1.0, bv = 0.0;
            int bp = 1 << 30;
            if (live) {
                double key = fabs(m[J]);
                if (key != key) key = -0.5;
                best = key;
                bp = t;
                bv = m[J];
            }
            argmax_step<kDppXor1>(best, bp, bv);
            argmax_step<kDppXor2>(best, bp, bv);
            argmax_step<0x124>(best, bp, bv);
            argmax_step<kDppRowRor8>(best, bp, bv);
            // the four 16-lane rows' winners, lowest position first on ties
#pragma unroll
            for (int rr = 1; rr < 4; ++rr) {
                const double ok = wave_bcast(best, 16 * rr);
                const int op = __builtin_amdgcn_readlane(bp, 16 * rr);
                const double ov = wave_bcast(bv, 16 * rr);
                argmax_take(best, bp, bv, ok, op, ov);
            }
            best = wave_bcast(best, 0);
            bp = __builtin_amdgcn_readfirstlane(bp);
            bv = wave_bcast(bv, 0);
            constexpr int R = 63 - J;
            if (t == bp) {
#pragma unroll
                for (int q = 0; q < R; ++q) sm.prow[w][par][J + 1 + q] = m[J + 1 + q];
            }
            if (lane == 0) {
                sm.key[w][par] = best;
                sm.val[w][par] = bv;
                sm.pos[w][par] = bp;
            }
            __syncthreads();
            const double k1 = sm.key[1][par];
            const int p1 = sm.pos[1][par];
            const double v1 = sm.val[1][par];
            double kb = sm.key[0][par], vb = sm.val[0][par];
            int pb = sm.pos[0][par];
            argmax_take(kb, pb, vb, k1, p1, v1);
            const int src = pb >> 6;
            if (t == 0) sm.sel[J] = pb;
            const double rv = (vb != 0.0) ? 1.0 / vb : 0.0;
            const bool upd = live && t != pb;
            const double l = upd ? m[J] * rv : 0.0;
            if (t == pb) live = false;
            // the pivot row in batches of at most 32 entries (registers)
            const double *pr = sm.prow[src][par];
            constexpr int R1 = R < 32 ? R : 32, R2 = R - R1;
            if constexpr (R1 > 0) {
                double cv[R1];
#pragma unroll
                for (int q = 0; q < R1; ++q) cv[q] = pr[J + 1 + q];
#pragma unroll
                for (int q = 0; q < R1; ++q) asm volatile("" : "+v"(cv[q]));
#pragma unroll
                for (int q = 0; q < R1; ++q) m[J + 1 + q] = fma(-l, cv[q], m[J + 1 + q]);
            }
            if constexpr (R2 > 0) {
                double cv[R2];
#pragma unroll
                for (int q = 0; q < R2; ++q) cv[q] = pr[J + 1 + R1 + q];
#pragma unroll
                for (int q = 0; q < R2; ++q) asm volatile("" : "+v"(cv[q]));
#pragma unroll
                for (int q = 0; q < R2; ++q) m[J + 1 + R1 + q] = fma(-l, cv[q], m[J + 1 + R1 + q]);
            }
        }
        TreeSelStep<J + 1>::run(sm, m, live, b);
    }
};
template <>
struct TreeSelStep<64> {
    __device__ __forceinline__ static void run(TreeSelSmem &, double (&)[64], bool &, int) {}
};

__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_tslu_tree(const double *__restrict__ A, int64_t lda, PanelArgs pa, TreeArgs ta, int b,
                 int32_t *__restrict__ cand) {
    __shared__ TreeSelSmem sm;
    const int64_t g = blockIdx.x;
    const int64_t left = (g / ta.width) * ta.span + g % ta.width;
    if (left >= pa.P) return;
    const int t = threadIdx.x;
    for (int64_t q = 1; q * ta.stride < ta.span && left + q * ta.stride < pa.P; ++q) {
        const int64_t right = left + q * ta.stride;
        if (t < 2 * b) sm.gidx[t] = (t < b) ? cand[left * b + t] : cand[right * b + (t - b)];
        __syncthreads();
        bool live = t < 2 * b;
        const double *src = A + (live ? sm.gidx[t] : 0);
        double m[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) m[k] = (live && k < b) ? src[(int64_t)k * lda] : 0.0;
        TreeSelStep<0>::run(sm, m, live, b);
        __syncthreads();
        if (t < b) cand[left * b + t] = sm.gidx[sm.sel[t]];
        __syncthreads();
    }
}

// U and the unit lower L11 of A[ipiv, :] by elimination without pivoting:
// thread i owns row i; row j is final after step j - 1.  info: the first
// zero U_jj (1-based), else 0.
// Step J of the no-pivot LU of the pivot block: lane i holds row i in m;
// lane J publishes row J's entries past J in LDS (double-buffered by step
// parity) and every lane reads them back in one batch (all loads issued
// before the first use); rows below J divide by the pivot and update their
// entries past J.  A zero pivot skips the step and records info.  Unrolled
// by template recursion so that every register index is a constant.
template <int J>
struct NoPivotStep {
    __device__ static void run(double (&m)[64], double (&row)[2][64], int i, int b, int &info) {
        if (J < b) {
            const double piv = wave_bcast(m[J], J);
            if (piv == 0.0) {
                if (!info) info = J + 1;
            } else {
                constexpr int R = 63 - J;
                if (i == J) {
#pragma unroll
                    for (int q = 0; q < R; ++q) row[J & 1][J + 1 + q] = m[J + 1 + q];
                }
                __syncthreads();
                const bool below = i > J && i < b;
                const double l = below ? m[J] / piv : 0.0;
                if (below) m[J] = l;
                if constexpr (R > 0) {
                    double cv[R];
#pragma unroll
                    for (int q = 0; q < R; ++q) cv[q] = row[J & 1][J + 1 + q];
#pragma unroll
                    for (int q = 0; q < R; ++q) asm volatile("" : "+v"(cv[q]));
                    if (below) {
#pragma unroll
                        for (int q = 0; q < R; ++q) m[J + 1 + q] = fma(-l, cv[q], m[J + 1 + q]);
                    }
                }
            }
        }
        NoPivotStep<J + 1>::run(m, row, i, b, info);
    }
};
template <>
struct NoPivotStep<64> {
    __device__ static void run(double (&)[64], double (&)[2][64], int, int, int &) {}
};

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_tslu_u(const double *__restrict__ A, int64_t lda, int b, const int32_t *__restrict__ cand,
              int64_t *__restrict__ ipiv, double *__restrict__ U, int64_t ldu, double *__restrict__ L11,
              int32_t *__restrict__ dinfo) {
    __shared__ double row[2][64];
    const int i = threadIdx.x;
    const int32_t gi = (i < b) ? cand[i] : 0;
    if (i < b) ipiv[i] = gi;
    double m[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) m[k] = (i < b && k < b) ? A[gi + (int64_t)k * lda] : 0.0;
    int info = 0;
    NoPivotStep<0>::run(m, row, i, b, info);
    if (i < b) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            if (k < b) {
                U[i + (int64_t)k * ldu] = (i <= k) ? m[k] : 0.0;
                L11[i + (int64_t)k * 64] = (k < i) ? m[k] : (k == i ? 1.0 : 0.0);
            }
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
        hipLaunchKernelGGL(k_tslu_tree, dim3((unsigned)ta.chains), dim3(128), 0, st, A, lda, pa, ta, b, cand);
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
