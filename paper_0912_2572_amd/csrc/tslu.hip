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
//                 the TSQR leaf's chunks, one thread per stack row;
//   k_tslu_tree   one workgroup per chain of a tree level (the TSQR tree's
//                 shapes): the left's candidates stacked on each right's,
//                 one thread per stack row (two waves);
//   k_tslu_u      U and the unit lower L11 of A[ipiv, :] without pivoting;
//   k_tslu_l      l_i = a_i U^{-1} for every row (one row per thread);
//   k_tslu_scatter  rows ipiv[k] of L <- row k of L11.
//
// Stack layout: thread t holds stack position t (row gidx[t] of A), its b
// entries in registers; a 256-row stack takes four waves, a tree node's
// 2b-row stack two.  An elimination step: each wave's pivot search by DPP
// and lane reads, the waves' winners (key, position, value and the pivot
// row past the step's column) through LDS with one barrier, then every
// live row's multiplier and the update of its entries past the column, the
// pivot row read back in batches of 32 entries.
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace tsqr {

namespace {

constexpr int kStack = 256;

// (value, position) pairs: the larger value wins, equal values go to the
// lower position.
__device__ __forceinline__ void argmax_take(double &best, int &bp, double &bv, double ob, int op, double ov) {
    if (ob > best || (ob == best && op < bp)) {
        best = ob;
        bp = op;
        bv = ov;
    }
}

// (best, bp, bv) of lanes l and l ^ 16 (permlane16_swap returns both of a
// pair's values to each lane), the better kept by both.
__device__ __forceinline__ void argmax_swap16(double &best, int &bp, double &bv) {
    const auto kl = __builtin_amdgcn_permlane16_swap(__double2loint(best), __double2loint(best), false, false);
    const auto kh = __builtin_amdgcn_permlane16_swap(__double2hiint(best), __double2hiint(best), false, false);
    const auto pp = __builtin_amdgcn_permlane16_swap(bp, bp, false, false);
    const auto vl = __builtin_amdgcn_permlane16_swap(__double2loint(bv), __double2loint(bv), false, false);
    const auto vh = __builtin_amdgcn_permlane16_swap(__double2hiint(bv), __double2hiint(bv), false, false);
    double k0 = __hiloint2double(kh[0], kl[0]), k1 = __hiloint2double(kh[1], kl[1]);
    double v0 = __hiloint2double(vh[0], vl[0]), v1 = __hiloint2double(vh[1], vl[1]);
    int p0 = (int)pp[0], p1 = (int)pp[1];
    asm volatile("" : "+v"(k0), "+v"(k1), "+v"(v0), "+v"(v1), "+v"(p0), "+v"(p1));
    best = k0;
    bp = p0;
    bv = v0;
    argmax_take(best, bp, bv, k1, p1, v1);
}
// The same for lanes l and l ^ 32.
__device__ __forceinline__ void argmax_swap32(double &best, int &bp, double &bv) {
    const auto kl = __builtin_amdgcn_permlane32_swap(__double2loint(best), __double2loint(best), false, false);
    const auto kh = __builtin_amdgcn_permlane32_swap(__double2hiint(best), __double2hiint(best), false, false);
    const auto pp = __builtin_amdgcn_permlane32_swap(bp, bp, false, false);
    const auto vl = __builtin_amdgcn_permlane32_swap(__double2loint(bv), __double2loint(bv), false, false);
    const auto vh = __builtin_amdgcn_permlane32_swap(__double2hiint(bv), __double2hiint(bv), false, false);
    double k0 = __hiloint2double(kh[0], kl[0]), k1 = __hiloint2double(kh[1], kl[1]);
    double v0 = __hiloint2double(vh[0], vl[0]), v1 = __hiloint2double(vh[1], vl[1]);
    int p0 = (int)pp[0], p1 = (int)pp[1];
    asm volatile("" : "+v"(k0), "+v"(k1), "+v"(v0), "+v"(v1), "+v"(p0), "+v"(p1));
    best = k0;
    bp = p0;
    bv = v0;
    argmax_take(best, bp, bv, k1, p1, v1);
}

// The lane exchanges below run on the whole wave before any comparison:
// empty asm statements keep the compiler from moving them into the
// conditional assignments, where they would read lanes that are off.
template <int CTRL>
__device__ __forceinline__ void argmax_step(double &best, int &bp, double &bv) {
    double ob = dpp_f64<CTRL>(best), ov = dpp_f64<CTRL>(bv);
    int op = __builtin_amdgcn_update_dpp(0, bp, CTRL, 0xf, 0xf, false);
    asm volatile("" : "+v"(ob), "+v"(op), "+v"(ov));
    argmax_take(best, bp, bv, ob, op, ov);
}

// Step J of partial-pivoting elimination on a stack of W waves, one thread
// per stack row, the row's entries in m:
//   each wave's argmax of |a_iJ| over its live rows (a NaN ranks below
//   every number, ties go to the lower stack position) by DPP inside each
//   16-lane row and lane-pair exchanges across the rows; the wave's winner puts
//   its row past J in LDS (one buffer per wave, double-buffered by step
//   parity) with its key; one barrier; every thread takes the best of the W
//   winners, reads that row back and updates its entries past J with
//   l = a_iJ * (1 / a_pJ) (one reciprocal: the multipliers only steer the
//   selection; U and L are computed from the chosen rows afterwards); a
//   zero pivot eliminates nothing.
template <int W>
struct RowSelSmem {
    double prow[W][2][64];   // [wave][parity][column]
    double key[W][2];        // [wave][parity]
    double val[W][2];
    int32_t pos[W][2];
    int32_t gidx[64 * W];
    int32_t sel[64];
};

template <int W, int J>
struct RowSelStep {
    __device__ __forceinline__ static void run(RowSelSmem<W> &sm, double (&m)[64], bool &live, int b) {
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
            // the four 16-lane rows' winners: rows 0|1 and 2|3 exchanged, then
            // the two halves (the take is symmetric, so every lane ends with
            // the wave's winner)
            argmax_swap16(best, bp, bv);
            argmax_swap32(best, bp, bv);
            bp = __builtin_amdgcn_readfirstlane(bp);
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
            double kb = sm.key[0][par], vb = sm.val[0][par];
            int pb = sm.pos[0][par];
#pragma unroll
            for (int u = 1; u < W; ++u) argmax_take(kb, pb, vb, sm.key[u][par], sm.pos[u][par], sm.val[u][par]);
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
        RowSelStep<W, J + 1>::run(sm, m, live, b);
    }
};
template <int W>
struct RowSelStep<W, 64> {
    __device__ __forceinline__ static void run(RowSelSmem<W> &, double (&)[64], bool &, int) {}
};

// One stack of `rows` rows (sm.gidx) on W waves, one thread per row: the
// kb = min(b, rows) selection steps, then gidx[0 .. kb-1] <- the chosen
// rows in pivot order.  Returns kb.
template <int W>
__device__ __forceinline__ int select_stack(RowSelSmem<W> &sm, const double *__restrict__ A, int64_t lda,
                                            int rows, int b) {
    const int t = threadIdx.x;
    bool live = t < rows;
    const double *src = A + (live ? sm.gidx[t] : 0);
    double m[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) m[k] = (live && k < b) ? src[(int64_t)k * lda] : 0.0;
    const int kb = b < rows ? b : rows;
    RowSelStep<W, 0>::run(sm, m, live, kb);
    __syncthreads();
    const int32_t g = (t < kb) ? sm.gidx[sm.sel[t]] : 0;
    __syncthreads();
    if (t < kb) sm.gidx[t] = g;
    return kb;
}

}  // namespace

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_tslu_leaf(const double *__restrict__ A, int64_t lda, PanelArgs pa, int b, int32_t *__restrict__ cand) {
    __shared__ RowSelSmem<4> sm;
    const int64_t dom = blockIdx.x;
    const int64_t row0 = dom_row0(pa, dom), end = row0 + dom_rows(pa, dom);
    const int t = threadIdx.x;
    int64_t pos = row0;
    int nc = 0;
    while (pos < end) {
        const int room = kStack - (nc ? b : 0);
        const int take = (int)((end - pos < room) ? end - pos : room);
        if (t >= nc && t < nc + take) sm.gidx[t] = (int32_t)(pos + (t - nc));
        __syncthreads();
        nc = select_stack<4>(sm, A, lda, nc + take, b);
        pos += take;
        __syncthreads();
    }
    if (t < b) cand[dom * b + t] = sm.gidx[t];
}

__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_tslu_tree(const double *__restrict__ A, int64_t lda, PanelArgs pa, TreeArgs ta, int b,
                 int32_t *__restrict__ cand) {
    __shared__ RowSelSmem<2> sm;
    const int64_t g = blockIdx.x;
    const int64_t left = (g / ta.width) * ta.span + g % ta.width;
    if (left >= pa.P) return;
    const int t = threadIdx.x;
    for (int64_t q = 1; q * ta.stride < ta.span && left + q * ta.stride < pa.P; ++q) {
        const int64_t right = left + q * ta.stride;
        if (t < 2 * b) sm.gidx[t] = (t < b) ? cand[left * b + t] : cand[right * b + (t - b)];
        __syncthreads();
        select_stack<2>(sm, A, lda, 2 * b, b);
        if (t < b) cand[left * b + t] = sm.gidx[t];
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
    {
        // every load in flight before the LDS stores
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = threadIdx.x + 256 * u, r = e & 63, c = e >> 6;
            v[u] = (r < b && c < b) ? U[r + (int64_t)c * ldu] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) Us[threadIdx.x + 256 * u] = v[u];
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
