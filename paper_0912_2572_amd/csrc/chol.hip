// chol.hip -- Cholesky factorization A = L L^T of a symmetric positive
// definite matrix, the third one-sided factorization the paper's
// introduction and conclusion carry the approach over to.
//
// Blocked right-looking Cholesky.  Block columns of kOuter = 256 columns;
// inside one, panels of kPanel = 64 columns:
//
//   k_chol_panel   per panel: the 64 x 64 diagonal block factored in one
//                  wave (lane t holds row t; l_jk reaches the other lanes by
//                  readlane), then every row below the block solved against
//                  it, l_i = a_i L11^{-T} (one wave per 64 rows, lane = row,
//                  L11 read from LDS as broadcasts).  Every workgroup
//                  factors the diagonal block itself, so one launch covers
//                  the panel;
//   k_chol_update  C -= W W^T on the lower triangle of a trailing block:
//                  with W the panel inside its block column (K = 64, the
//                  columns of the rest of the block column), then with W
//                  the whole block column (K = 256, the trailing matrix).
//                  FP64 matrix-core tiles over TILE x TILE output tiles of
//                  the lower triangle, operands staged through LDS in
//                  16-column chunks (double-buffered).
//
// The trailing matrix is read and written once per 256-column block
// column: with 128 x 128 tiles that is 2 x 8 bytes of HBM traffic per 2 x
// 256 flops, which keeps the update on the matrix cores' side of the
// roofline (the communication-avoiding blocking of the sequential Cholesky
// algorithms the paper cites).
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

__global__ __launch_bounds__(64) void k_chol_info_clear(int32_t *dinfo) {
    if (threadIdx.x == 0) *dinfo = 0;
}

// Panel of columns s .. s + sb - 1 (1 <= sb <= 64): the diagonal block
// (rows s .. s + sb - 1) and the rows s + sb + 64 blockIdx.x + lane.
// The factorization's steps take l_jk from lane j's registers (readlane);
// the row solve reads L11 from LDS, a column ahead of its use.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_chol_panel(double *__restrict__ A, int64_t lda, int64_t n, int64_t s, int sb,
                  int32_t *__restrict__ dinfo) {
    if (*(volatile int32_t *)dinfo != 0) return;
    // Lc[64 k + i] = L(i, k) of the diagonal block for i > k (rows >= sb are
    // zero) and 1 / L(k, k) at i = k
    __shared__ double Lc[kPanel * kPanel];
    const int t = threadIdx.x;
    double *__restrict__ Ad = A + s + s * lda;

    // Row t of the diagonal block, lower part (rows past sb stay zero).
    double m[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) m[j] = (j < sb && j <= t && t < sb) ? Ad[t + j * lda] : 0.0;

    // Right-looking factorization: step k finishes column k of L and updates
    // the columns after it.
    int fail = -1;
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        if (k >= sb || fail >= 0) continue;
        const double d = wave_bcast(m[k], k);
        if (!(d > 0.0)) {
            fail = k;
            continue;
        }
        const double ljj = sqrt(d);
        const double rinv = 1.0 / ljj;
        const double v = t < k ? 0.0 : (t == k ? ljj : m[k] * rinv);
        m[k] = v;
        Lc[kPanel * k + t] = t == k ? rinv : v;
#pragma unroll
        for (int j = k + 1; j < kPanel; ++j) m[j] = fma(-v, wave_bcast(v, j), m[j]);
    }
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

    // Rows below: x L11^T = a by forward substitution, lane = row.
    const int64_t r = s + sb + (int64_t)blockIdx.x * kPanel + t;
    if (r >= n) return;
    double *__restrict__ Ar = A + r + s * lda;
    double x[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) x[j] = j < sb ? Ar[j * lda] : 0.0;
    double c[2][kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) c[0][j] = Lc[j];
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
        if (k >= sb) continue;
        if (k + 1 < kPanel) {
#pragma unroll
            for (int j = k + 1; j < kPanel; ++j) c[(k + 1) & 1][j] = Lc[kPanel * (k + 1) + j];
        }
        const double xk = x[k] * c[k & 1][k];
        x[k] = xk;
#pragma unroll
        for (int j = k + 1; j < kPanel; ++j) x[j] = fma(-xk, c[k & 1][j], x[j]);
    }
#pragma unroll
    for (int j = 0; j < kPanel; ++j)
        if (j < sb) Ar[j * lda] = x[j];
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
            const int64_t grid = below > 0 ? (below + kPanel - 1) / kPanel : 1;
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
            // 128-row tiles once they give two workgroups per compute unit
            const int64_t T = (n - jend + 127) / 128;
            if (T * (T + 1) / 2 >= 2 * 256)
                e = update<128>(A, lda, n, jend, n, j, (int)(jend - j), dinfo, "chol_syrk", st);
            else
                e = update<64>(A, lda, n, jend, n, j, (int)(jend - j), dinfo, "chol_syrk", st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace tsqr
