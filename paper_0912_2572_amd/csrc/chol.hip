// chol.hip -- Cholesky factorization A = L L^T of a symmetric positive
// definite matrix, the third one-sided factorization the paper's
// introduction and conclusion carry the approach over to.
//
// Blocked right-looking Cholesky.  Block columns of kOuter = 256 columns;
// inside one, panels of kPanel = 64 columns:
//
//   k_chol_panel   per panel: the 64 x 64 diagonal block factored in one
//                  wave (lane t holds row t; column k of L goes through LDS
//                  and comes back to every lane as broadcasts), then every
//                  row below the block solved against it, l_i = a_i
//                  L11^{-T} (one wave per 32 rows, a lane pair per row
//                  splitting its columns by parity).  Every workgroup
//                  factors the diagonal block itself, so one launch covers
//                  the panel;
//   k_chol_update  C -= W W^T on the lower triangle of a trailing block:
//                  with W the panel inside its block column (K = 64, the
//                  columns of the rest of the block column), then with W
//                  the whole block column (K = 256, the trailing matrix).
//                  FP64 matrix-core tiles over 64 x 64 output tiles of
//                  the lower triangle, operands staged through LDS in
//                  16-column chunks (double-buffered).
//
// The trailing matrix is read and written once per 256-column block
// column: 2 x 8 bytes of HBM traffic per 2 x 256 flops, which keeps the
// update on the matrix cores' side of the roofline (the
// communication-avoiding blocking of the sequential Cholesky algorithms the
// paper cites); the operands, a 256-column block of L, are re-read from
// the caches by every tile.
//
// A failed pivot (<= 0 or NaN) writes j + 1 to the info word; every later
// kernel reads the word first and returns at once.
#include "common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

namespace {

constexpr int kPanel = 64;
constexpr int kOuter = 256;

// 1 / sqrt(d) for a positive normal d: the hardware estimate and two
// Newton steps r <- r (3/2 - d r^2 / 2), each squaring the relative error.
__device__ __forceinline__ double rsqrt_f64(double d) {
    double r = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    r = r * fma(-hd, r * r, 1.5);
    r = r * fma(-hd, r * r, 1.5);
    return r;
}

// The steps of the panel kernel, unrolled by template recursion so that
// every register index is a compile-time constant.  A step reads its
// column of L11 from LDS into registers and marks each value as used, in
// order, with an empty asm statement: every load is then issued before the
// first use instead of one load in front of each use.

// Column K of L11 in LDS: L(i, K), i != K, at lc_at(K, i) (the even rows,
// then the odd ones, so that a lane pair's halves are contiguous); 1 /
// L(K, K) at 64 * 64 + K.
__host__ __device__ constexpr int lc_at(int K, int i) { return kPanel * K + 32 * (i & 1) + (i >> 1); }

// Factorization step K: lane t holds row t of the diagonal block in m.
template <int K>
struct FactorStep {
    __device__ __forceinline__ static void run(double (&m)[kPanel], double *Lc, int t, int sb, int &fail) {
        if (K < sb && fail < 0) {
            const double d = wave_bcast(m[K], K);
            if (!(d > 0.0)) {
                fail = K;
            } else {
                const double rinv = rsqrt_f64(d);
                const double v = t < K ? 0.0 : (t == K ? d * rinv : m[K] * rinv);
                m[K] = v;
                if (t == K) Lc[kPanel * kPanel + K] = rinv;
                else Lc[lc_at(K, t)] = v;
                __syncthreads();
                constexpr int R = kPanel - K - 1;
                if constexpr (R > 0) {
                    double cv[R];
#pragma unroll
                    for (int i = 0; i < R; ++i) cv[i] = Lc[lc_at(K, K + 1 + i)];
#pragma unroll
                    for (int i = 0; i < R; ++i) asm volatile("" : "+v"(cv[i]));
#pragma unroll
                    for (int i = 0; i < R; ++i) m[K + 1 + i] = fma(-v, cv[i], m[K + 1 + i]);
                }
            }
        }
        FactorStep<K + 1>::run(m, Lc, t, sb, fail);
    }
};
template <>
struct FactorStep<kPanel> {
    __device__ __forceinline__ static void run(double (&)[kPanel], double *, int, int, int &) {}
};

// Solve step K on a lane pair: lane h = lane & 1 of the pair holds the
// columns j = 2 q + h of its row in xh[q].  The owner of column K (h = K & 1)
// forms x_K = x_K / L(K, K) and passes it to its partner by DPP; each lane
// then updates its columns past K with column K of L11, its half read from
// LDS in one batch.
template <int K>
struct PairSolveStep {
    __device__ __forceinline__ static void run(double (&xh)[kPanel / 2], const double *Lc, int h, int sb) {
        if (K < sb) {
            constexpr int hK = K & 1, qK = K >> 1, Q0 = K >> 1, R = kPanel / 2 - Q0;
            const double own = xh[qK] * Lc[kPanel * kPanel + K];
            // the exchange runs on the whole wave before the select (inside
            // a branch on the non-owners it would read lanes that are off)
            double other = dpp_f64<kDppXor1>(own);
            asm volatile("" : "+v"(other));
            const double xk = (h == hK) ? own : other;
            if (h == hK) xh[qK] = xk;
            double cv[R];
            const double *col = Lc + kPanel * K + 32 * h;
#pragma unroll
            for (int q = 0; q < R; ++q) cv[q] = col[Q0 + q];
#pragma unroll
            for (int q = 0; q < R; ++q) asm volatile("" : "+v"(cv[q]));
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (2 * (Q0 + q) + h > K) xh[Q0 + q] = fma(-xk, cv[q], xh[Q0 + q]);
        }
        PairSolveStep<K + 1>::run(xh, Lc, h, sb);
    }
};
template <>
struct PairSolveStep<kPanel> {
    __device__ __forceinline__ static void run(double (&)[kPanel / 2], const double *, int, int) {}
};

__global__ __launch_bounds__(64) void k_chol_info_clear(int32_t *dinfo) {
    if (threadIdx.x == 0) *dinfo = 0;
}

// Panel of columns s .. s + sb - 1 (1 <= sb <= 64): the diagonal block
// (rows s .. s + sb - 1) and the rows s + sb + 32 blockIdx.x + lane / 2.
// Both phases read a column of L11 from LDS as broadcasts, all of its
// loads issued before the first use.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_chol_panel(double *__restrict__ A, int64_t lda, int64_t n, int64_t s, int sb,
                  int32_t *__restrict__ dinfo) {
    if (*(volatile int32_t *)dinfo != 0) return;
    // column k of L11 at lc_at(k, i) (rows >= sb zero), 1 / L(k, k) at
    // 64 * 64 + k
    __shared__ double Lc[kPanel * kPanel + kPanel];
    const int t = threadIdx.x;
    double *__restrict__ Ad = A + s + s * lda;

    // Row t of the diagonal block, lower part (rows past sb stay zero).
    double m[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) m[j] = (j < sb && j <= t && t < sb) ? Ad[t + j * lda] : 0.0;

    // Right-looking factorization: step k finishes column k of L and updates
    // the columns after it.
    int fail = -1;
    FactorStep<0>::run(m, Lc, t, sb, fail);
    if (fail >= 0) {
        if (t == 0) *dinfo = (int32_t)(s + fail + 1);
        return;
    }
    if (blockIdx.x == 0 && t < sb) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j)
            if (j <= t) Ad[t + j * lda] = m[j];
    }
    __syncthreads();

    // Rows below: x L11^T = a by forward substitution, a lane pair per row
    // (32 rows per workgroup), lane h of the pair on the columns 2 q + h.
    const int h = t & 1;
    const int64_t r = s + sb + (int64_t)blockIdx.x * (kPanel / 2) + (t >> 1);
    const bool rok = r < n;
    double *__restrict__ Ar = A + (rok ? r : 0) + s * lda;
    double xh[kPanel / 2];
#pragma unroll
    for (int q = 0; q < kPanel / 2; ++q) xh[q] = (rok && 2 * q + h < sb) ? Ar[(2 * q + h) * lda] : 0.0;
    PairSolveStep<0>::run(xh, Lc, h, sb);
    if (!rok) return;
#pragma unroll
    for (int q = 0; q < kPanel / 2; ++q)
        if (2 * q + h < sb) Ar[(2 * q + h) * lda] = xh[q];
}

// C(i, c) -= sum_{k < K} A(i, kc + k) A(c, kc + k) for t0 <= c < cend,
// c <= i < n: the lower triangle of a trailing block, by TILE x TILE tiles
// (bi, bc), bc <= bi, numbered column after column.  Four waves in a 2 x 2
// grid of (TILE/2) x (TILE/2) sub-tiles.
template <int TILE>
__global__ __launch_bounds__(256) void k_chol_update(double *__restrict__ A, int64_t lda, int64_t n, int64_t t0,
                                                     int64_t cend, int64_t kc, int K, int64_t Tr, int64_t Tc,
                                                     const int32_t *__restrict__ dinfo) {
    if (*(const volatile int32_t *)dinfo != 0) return;
    constexpr int WT = TILE / 32;       // 16 x 16 tiles per wave and dimension
    constexpr int KSTEP = 256 / TILE;   // loader: k stride between one thread's loads
    constexpr int LPT = TILE / 16;      // loads per thread and operand per chunk
    static_assert(KSTEP * LPT == 16, "16-column chunks");
    __shared__ double As[2][16][TILE];
    __shared__ double Bs[2][16][TILE];

    // tile id -> (bi, bc): column bc starts at bc Tr - bc (bc - 1) / 2
    const int64_t id = blockIdx.x;
    int64_t lo = 0, hi = Tc - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (mid * Tr - mid * (mid - 1) / 2 <= id) lo = mid;
        else hi = mid - 1;
    }
    const int64_t bc = lo;
    const int64_t bi = bc + (id - (bc * Tr - bc * (bc - 1) / 2));
    const int64_t i0 = t0 + bi * TILE, c0 = t0 + bc * TILE;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;
    // on a diagonal tile the upper-right sub-tile is above the diagonal
    const bool idle = (bi == bc) && (wi < wj);

    const int lrow = tid % TILE, lk = tid / TILE;
    const int64_t ar = i0 + lrow, br = c0 + lrow;
    const bool aok = ar < n, bok = br < n;
    const double *__restrict__ Aa = A + (aok ? ar : 0) + kc * lda;
    const double *__restrict__ Ab = A + (bok ? br : 0) + kc * lda;

    d4 acc[WT][WT];
#pragma unroll
    for (int I = 0; I < WT; ++I)
#pragma unroll
        for (int J = 0; J < WT; ++J) acc[I][J] = d4_zero();

    double ra[LPT], rb[LPT];
    auto load = [&](int ch) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int k = 16 * ch + lk + KSTEP * q;
            ra[q] = (aok && k < K) ? Aa[k * lda] : 0.0;
            rb[q] = (bok && k < K) ? Ab[k * lda] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            As[buf][lk + KSTEP * q][lrow] = ra[q];
            Bs[buf][lk + KSTEP * q][lrow] = rb[q];
        }
    };

    const int nch = (K + 15) / 16;
    load(0);
    stash(0);
    __syncthreads();
    const int ri = wi * (TILE / 2) + (lane & 15), rj = wj * (TILE / 2) + (lane & 15);
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load(ch + 1);
        if (!idle) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 4 * ks + (lane >> 4);
                double a[WT], b[WT];
#pragma unroll
                for (int I = 0; I < WT; ++I) a[I] = As[buf][kk][ri + 16 * I];
#pragma unroll
                for (int J = 0; J < WT; ++J) b[J] = Bs[buf][kk][rj + 16 * J];
#pragma unroll
                for (int I = 0; I < WT; ++I)
#pragma unroll
                    for (int J = 0; J < WT; ++J) acc[I][J] = mfma_f64(a[I], b[J], acc[I][J]);
            }
        }
        if (ch + 1 < nch) stash(buf ^ 1);
        __syncthreads();
    }
    if (idle) return;

#pragma unroll
    for (int I = 0; I < WT; ++I)
#pragma unroll
        for (int J = 0; J < WT; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = i0 + wi * (TILE / 2) + 16 * I + d_row(r, lane);
                const int64_t col = c0 + wj * (TILE / 2) + 16 * J + d_col(lane);
                if (row < n && col < cend && row >= col) A[row + col * lda] -= acc[I][J][r];
            }
}

template <int TILE>
hipError_t update(double *A, int64_t lda, int64_t n, int64_t t0, int64_t cend, int64_t kc, int K,
                  const int32_t *dinfo, const char *tag, hipStream_t st) {
    const int64_t Tr = (n - t0 + TILE - 1) / TILE, Tc = (cend - t0 + TILE - 1) / TILE;
    const int64_t tiles = Tc * Tr - Tc * (Tc - 1) / 2;
    if (tiles <= 0) return hipSuccess;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    ProfScope ps(tag, st);
    hipLaunchKernelGGL(k_chol_update<TILE>, dim3((unsigned)tiles), dim3(256), 0, st, A, lda, n, t0, cend, kc, K,
                       Tr, Tc, dinfo);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cholesky(int64_t n, double *A, int64_t lda, int32_t *dinfo, hipStream_t st) {
    hipLaunchKernelGGL(k_chol_info_clear, dim3(1), dim3(64), 0, st, dinfo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int64_t j = 0; j < n; j += kOuter) {
        const int64_t jend = j + kOuter < n ? j + kOuter : n;
        for (int64_t s = j; s < jend; s += kPanel) {
            const int sb = (int)(jend - s < kPanel ? jend - s : kPanel);
            const int64_t below = n - s - sb;
            const int64_t grid = below > 0 ? (below + kPanel / 2 - 1) / (kPanel / 2) : 1;
            {
                ProfScope ps("chol_panel", st);
                hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)grid), dim3(kPanel), 0, st, A, lda, n, s, sb, dinfo);
                e = hipGetLastError();
            }
            if (e != hipSuccess) return e;
            if (s + sb < jend) {
                e = update<64>(A, lda, n, s + sb, jend, s, sb, dinfo, "chol_update", st);
                if (e != hipSuccess) return e;
            }
        }
        if (jend < n) {
            // 64 x 64 tiles: four resident workgroups per compute unit hide
            // the operand loads better than 128 x 128 tiles' reuse pays
            // (8192 x 8192: 4.8 against 6.4 ms of trailing updates)
            e = update<64>(A, lda, n, jend, n, j, (int)(jend - j), dinfo, "chol_syrk", st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace tsqr
