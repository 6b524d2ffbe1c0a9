// calu.hip -- LU of an m x n matrix (m >= n) with tournament pivoting
// (CALU), the LU counterpart of CAQR that the paper's conclusion names
// beside TSLU.  Panels of 64 columns; panel k:
//
//   TSLU (tslu.hip) of the m - k rows below the diagonal: the tournament's
//     pivot rows, U11 and L = A U11^{-1} in the panel's row order;
//   k_calu_swaps   one wave turns the pivot rows into LAPACK-style row
//                  interchanges (interchange i swaps rows k + i and
//                  k + swp[i], swp[i] = where the i-th pivot row sits after
//                  interchanges 0..i-1) and merges the panel's info word;
//   k_calu_rowswap the interchanges on every column outside the panel, as
//                  one gather per column over the touched positions;
//   k_calu_pack    the panel's columns in the permuted row order: U on and
//                  above the diagonal block's diagonal, L below (row rel
//                  takes the L row of the original row that the interchanges
//                  brought there);
//   k_calu_trsm    U12 = L11^{-1} A12 by forward substitution (unit
//                  diagonal), one thread per column, L11 in LDS;
//   k_lu_update    A22 -= L21 U12 on the FP64 matrix cores, 64 x 64 tiles,
//                  operands staged through LDS in 16-deep chunks.
#include "common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

namespace {

constexpr int kLuPanel = 64;

// Per-panel interchange record (int32 words): swp[0..63], then the touched
// positions (at most 128: the top b and the displaced ones), the row each
// ends up holding (its position before the panel's interchanges), and their
// count.
constexpr int kMetaSwp = 0, kMetaPos = 64, kMetaSrc = 192, kMetaCount = 320;

__global__ __launch_bounds__(64) void k_calu_clear(int32_t *dinfo) {
    if (threadIdx.x == 0) *dinfo = 0;
}

// swp[i] from the pivot rows piv (relative to row k), on one wave.  Lane t
// tracks the row at position t < b (top) and one position at or past b that
// an interchange has filled with another row (the displaced list, nd
// entries); every other position holds its own row.  Step i finds where
// piv[i] sits by a ballot over both, exchanges it with position i and
// records the row it displaces.  ipiv_out[i] = k + swp[i].  The touched
// positions and the rows they end up holding go to meta (see CaluMeta) for
// the row exchange.  dinfo <- k + pinfo on the first panel whose U has an
// exactly zero diagonal entry.
__global__ __launch_bounds__(64) void k_calu_swaps(const int64_t *__restrict__ piv, int b, int64_t k,
                                                   int32_t *__restrict__ meta, int64_t *__restrict__ ipiv_out,
                                                   const int32_t *__restrict__ pinfo, int32_t *__restrict__ dinfo) {
    int32_t *__restrict__ swp = meta + kMetaSwp;
    const int t = threadIdx.x;
    __shared__ int64_t pv[kLuPanel];
    if (t < b) pv[t] = piv[t];
    __syncthreads();
    int64_t top = t, dpos = -1, drow = -1;
    int nd = 0;
    int64_t mine = 0;   // swp[t], kept by lane t
    for (int i = 0; i < b; ++i) {
        const int64_t r = pv[i];
        const uint64_t m1 = __ballot(t >= i && t < b && top == r);
        const uint64_t m2 = __ballot(t < nd && drow == r);
        int64_t p;
        int dl = -1;
        if (m1) {
            p = __builtin_ctzll(m1);
        } else if (m2) {
            dl = __builtin_ctzll(m2);
            const int64_t dp = dpos;
            p = (int64_t)__shfl(dp, dl);
        } else {
            p = r;
        }
        const int64_t tp = top;
        const int64_t ri = __shfl(tp, i);   // the row at position i, displaced to p
        if (t == i) {
            top = r;
            mine = p;
        }
        if (p < b) {
            if (t == p && p != i) top = ri;
        } else if (dl >= 0) {
            if (t == dl) drow = ri;
        } else {
            if (t == nd) {
                dpos = p;
                drow = ri;
            }
            ++nd;
        }
    }
    if (t < b) {
        swp[t] = (int32_t)mine;
        ipiv_out[t] = k + mine;
        meta[kMetaPos + t] = t;
        meta[kMetaSrc + t] = (int32_t)top;
    }
    if (t < nd) {
        meta[kMetaPos + b + t] = (int32_t)dpos;
        meta[kMetaSrc + b + t] = (int32_t)drow;
    }
    if (t == 0) meta[kMetaCount] = b + nd;
    if (t == 0) {
        const int32_t pi = *pinfo;
        if (pi > 0 && *dinfo == 0) *dinfo = (int32_t)(k + pi);
    }
}

// Columns outside [k, k + b): the interchanges as one gather per column
// (the touched positions take the rows recorded for them; all loads of a
// column are issued before its stores).  Four columns per workgroup, one
// wave each, two touched positions per lane.
__global__ __launch_bounds__(256) void k_calu_rowswap(double *__restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                      int b, const int32_t *__restrict__ meta) {
    const int lane = threadIdx.x & 63;
    int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int cnt = meta[kMetaCount];
    const bool live = c < n - b;
    if (c >= k) c += b;
    double *col = A + (live ? c : 0) * lda + k;
    const bool q0 = live && lane < cnt, q1 = live && lane + 64 < cnt;
    const int p0 = q0 ? meta[kMetaPos + lane] : 0, p1 = q1 ? meta[kMetaPos + lane + 64] : 0;
    const double v0 = q0 ? col[meta[kMetaSrc + lane]] : 0.0;
    const double v1 = q1 ? col[meta[kMetaSrc + lane + 64]] : 0.0;
    __syncthreads();
    if (q0) col[p0] = v0;
    if (q1) col[p1] = v1;
}

// Panel columns, row rel = 0 .. mr - 1 below row k: the original row o that
// the interchanges brought to rel (walk them backwards), then U11[rel][j]
// for rel < b, j >= rel, else L[o][j] (L: mr x b, ld ldl).
__global__ __launch_bounds__(256) void k_calu_pack(double *__restrict__ A, int64_t lda, int64_t mr, int64_t k,
                                                   int b, const int32_t *__restrict__ meta,
                                                   const double *__restrict__ L, int64_t ldl,
                                                   const double *__restrict__ U, int64_t ldu) {
    __shared__ int32_t s[kLuPanel];
    if (threadIdx.x < b) s[threadIdx.x] = meta[kMetaSwp + threadIdx.x];
    __syncthreads();
    const int64_t rel = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rel >= mr) return;
    int64_t o = rel;
    for (int i = b - 1; i >= 0; --i) {
        if (o == i) o = s[i];
        else if (o == s[i]) o = i;
    }
    double *dst = A + (k + rel) + k * lda;
    double v[kLuPanel];
#pragma unroll
    for (int j = 0; j < kLuPanel; ++j)
        v[j] = (j < b) ? ((rel < b && j >= rel) ? U[rel + j * ldu] : L[o + j * ldl]) : 0.0;
#pragma unroll
    for (int j = 0; j < kLuPanel; ++j)
        if (j < b) dst[j * lda] = v[j];
}

// Step L of the unit-lower forward substitution: y[i] -= y[L] L11(i, L),
// i > L, with column L of L11 read from LDS into registers, every load
// issued before the first use (empty asm statements mark the values used
// in order).  Unrolled by template recursion: every index is a constant.
template <int L>
struct UnitSolveStep {
    __device__ static void run(double (&y)[kLuPanel], const double *Ls, int b) {
        if (L < b) {
            constexpr int R = kLuPanel - L - 1;
            if constexpr (R > 0) {
                double cv[R];
#pragma unroll
                for (int i = 0; i < R; ++i) cv[i] = Ls[kLuPanel * L + L + 1 + i];
#pragma unroll
                for (int i = 0; i < R; ++i) asm volatile("" : "+v"(cv[i]));
#pragma unroll
                for (int i = 0; i < R; ++i) y[L + 1 + i] = fma(-y[L], cv[i], y[L + 1 + i]);
            }
        }
        UnitSolveStep<L + 1>::run(y, Ls, b);
    }
};
template <>
struct UnitSolveStep<kLuPanel> {
    __device__ static void run(double (&)[kLuPanel], const double *, int) {}
};

// U12 = L11^{-1} A12 for columns c in [k + b, n): one thread per column,
// L11 (unit lower, rows/columns k .. k + b - 1 of the packed A) in LDS.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_calu_trsm(double *__restrict__ A, int64_t lda, int64_t n, int64_t k, int b) {
    __shared__ double Ls[kLuPanel * kLuPanel];   // Ls[64 l + i] = L11(i, l)
    const int t = threadIdx.x;
    {
        // every load in flight before the LDS stores
        double v[kLuPanel];
#pragma unroll
        for (int l = 0; l < kLuPanel; ++l) v[l] = (t < b && l < b) ? A[(k + t) + (k + l) * lda] : 0.0;
#pragma unroll
        for (int l = 0; l < kLuPanel; ++l)
            if (l < b) Ls[kLuPanel * l + t] = v[l];
    }
    __syncthreads();
    const int64_t c = k + b + (int64_t)blockIdx.x * kLuPanel + t;
    if (c >= n) return;
    double *col = A + c * lda + k;
    double y[kLuPanel];
#pragma unroll
    for (int i = 0; i < kLuPanel; ++i) y[i] = i < b ? col[i] : 0.0;
    UnitSolveStep<0>::run(y, Ls, b);
#pragma unroll
    for (int i = 0; i < kLuPanel; ++i)
        if (i < b) col[i] = y[i];
}

// A(i, c) -= sum_{kk < K} A(i, k + kk) A(k + kk, c) for i in [r0, m),
// c in [r0, n), r0 = k + K: 64 x 64 tiles (bi = id mod Tr, bc = id / Tr),
// four waves in a 2 x 2 grid of 32 x 32 sub-tiles.
__global__ __launch_bounds__(256) void k_lu_update(double *__restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                   int64_t k, int K, int64_t Tr) {
    constexpr int TILE = 64, WT = 2;
    __shared__ double As[2][16][TILE];
    __shared__ double Bs[2][16][TILE];
    const int64_t r0 = k + K;
    const int64_t bi = (int64_t)blockIdx.x % Tr, bc = (int64_t)blockIdx.x / Tr;
    const int64_t i0 = r0 + bi * TILE, c0 = r0 + bc * TILE;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;

    // A operand: row i0 + (tid & 63), depth (tid >> 6) + 4 q; B operand:
    // depth tid & 15 (16 consecutive rows of U12), column c0 + (tid >> 4) + 16 q
    const int arow = tid & 63, ak = tid >> 6;
    const int bk = tid & 15, bcol = tid >> 4;
    const bool aok = i0 + arow < m;
    const double *__restrict__ Aa = A + (aok ? i0 + arow : 0) + k * lda;
    double ra[4], rb[4];
    auto load = [&](int ch) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = 16 * ch + ak + 4 * q;
            ra[q] = (aok && kk < K) ? Aa[kk * lda] : 0.0;
            const int kb = 16 * ch + bk;
            const int64_t c = c0 + bcol + 16 * q;
            rb[q] = (kb < K && c < n) ? A[(k + kb) + c * lda] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][ak + 4 * q][arow] = ra[q];
            Bs[buf][bk][bcol + 16 * q] = rb[q];
        }
    };
    d4 acc[WT][WT];
#pragma unroll
    for (int I = 0; I < WT; ++I)
#pragma unroll
        for (int J = 0; J < WT; ++J) acc[I][J] = d4_zero();
    const int nch = (K + 15) / 16;
    load(0);
    stash(0);
    __syncthreads();
    const int ri = wi * (TILE / 2) + (lane & 15), rj = wj * (TILE / 2) + (lane & 15);
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load(ch + 1);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = 4 * ks + (lane >> 4);
            double a[WT], bv[WT];
#pragma unroll
            for (int I = 0; I < WT; ++I) a[I] = As[buf][kk][ri + 16 * I];
#pragma unroll
            for (int J = 0; J < WT; ++J) bv[J] = Bs[buf][kk][rj + 16 * J];
#pragma unroll
            for (int I = 0; I < WT; ++I)
#pragma unroll
                for (int J = 0; J < WT; ++J) acc[I][J] = mfma_f64(a[I], bv[J], acc[I][J]);
        }
        if (ch + 1 < nch) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int I = 0; I < WT; ++I)
#pragma unroll
        for (int J = 0; J < WT; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = i0 + wi * (TILE / 2) + 16 * I + d_row(r, lane);
                const int64_t col = c0 + wj * (TILE / 2) + 16 * J + d_col(lane);
                if (row < m && col < n) A[row + col * lda] -= acc[I][J][r];
            }
}

}  // namespace

hipError_t launch_calu_clear(int32_t *dinfo, hipStream_t st) {
    hipLaunchKernelGGL(k_calu_clear, dim3(1), dim3(64), 0, st, dinfo);
    return hipGetLastError();
}

hipError_t launch_calu_panel_rest(double *A, int64_t lda, int64_t m, int64_t n, int64_t k, int b,
                                  const int64_t *piv, int32_t *meta, int64_t *ipiv_out, const int32_t *pinfo,
                                  int32_t *dinfo, const double *L, int64_t ldl, const double *U, int64_t ldu,
                                  hipStream_t st) {
    if (b < 1 || b > kLuPanel) return hipErrorInvalidValue;
    {
        ProfScope ps("calu_swaps", st);
        hipLaunchKernelGGL(k_calu_swaps, dim3(1), dim3(64), 0, st, piv, b, k, meta, ipiv_out + k, pinfo, dinfo);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n > b) {
        ProfScope ps("calu_rowswap", st);
        hipLaunchKernelGGL(k_calu_rowswap, dim3((unsigned)((n - b + 3) / 4)), dim3(256), 0, st, A, lda, n, k, b,
                           meta);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        ProfScope ps("calu_pack", st);
        const int64_t mr = m - k;
        hipLaunchKernelGGL(k_calu_pack, dim3((unsigned)((mr + 255) / 256)), dim3(256), 0, st, A, lda, mr, k, b,
                           meta, L, ldl, U, ldu);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (k + b < n) {
        {
            ProfScope ps("calu_trsm", st);
            const int64_t cols = n - k - b;
            hipLaunchKernelGGL(k_calu_trsm, dim3((unsigned)((cols + kLuPanel - 1) / kLuPanel)), dim3(kLuPanel), 0,
                               st, A, lda, n, k, b);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const int64_t Tr = (m - k - b + 63) / 64, Tc = (n - k - b + 63) / 64;
        if (Tr * Tc > INT32_MAX) return hipErrorInvalidValue;
        ProfScope ps("calu_update", st);
        hipLaunchKernelGGL(k_lu_update, dim3((unsigned)(Tr * Tc)), dim3(256), 0, st, A, lda, m, n, k, b, Tr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tsqr
