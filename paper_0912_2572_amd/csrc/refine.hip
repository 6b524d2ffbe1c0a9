// refine.hip -- mixed-precision support: FP32 copies of the reflectors and
// the FP64 pieces of least-squares iterative refinement.
//
// With the mixed factor Q~ R~ (FP32 WY applies), least squares is brought
// back to FP64 accuracy by refining the augmented system
//     [ I   A ] [r]   [b]
//     [ A^T 0 ] [x] = [0]
// (Bjorck's method): with FP64 residuals f = b - r - A x and g = -A^T r, the
// correction solves through the factors are
//     R^T h = g,   d = Q^T f,   dx = R^{-1} (d_1 - h),   dr = Q [h; d_2],
// and x += dx, r += dr.  Plain x-only refinement would stall at the
// accuracy of the FP32 factor for problems with a large residual; the
// augmented form does not.  The paper fixes only the QR (Sec. 2.2) and
// names least squares as its use; the refinement is the textbook one.
#include "common.h"
#include "kernels.h"
#include "plan.h"
#include "prof.h"

namespace tsqr {

__global__ void k_to_f32(const double *__restrict__ src, int64_t lds, float *__restrict__ dst, int64_t ldd,
                         int64_t rows, int64_t cols) {
    const int64_t total = rows * cols;
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < total;
         e += (int64_t)blockDim.x * gridDim.x) {
        const int64_t r = e % rows, c = e / rows;
        dst[r + c * ldd] = (float)src[r + c * lds];
    }
}

constexpr int kResRows = 32;   // rows per LDS tile of the residual pass

// One pass over A (FP64): F = B - Rr - A X (rows of this block),
// gpart[block] = A_block^T Rr_block (n x k), and rpart[block] = the squared
// column norms of (B - A X)_block (entries 0..k-1) and of F_block (entries
// k..2k-1), all in a fixed summation order.
__device__ __forceinline__ void resid_block(const double *__restrict__ A, int64_t lda, int64_t m, int n,
                                            const double *__restrict__ B, int64_t ldb,
                                            const double *__restrict__ X, int64_t ldx,
                                            const double *__restrict__ Rr, double *__restrict__ F, int k,
                                            double *__restrict__ gpart, double *__restrict__ rpart,
                                            int64_t blk, int64_t nblk, double *sh) {
    double *At = sh;                        // kResRows x n (row-major)
    double *Xs = At + kResRows * n;         // n x k
    double *Rt = Xs + n * k;                // kResRows x k
    double *Ss = Rt + kResRows * k;         // kResRows x k: (B - A X)^2
    double *Fs = Ss + kResRows * k;         // kResRows x k: F^2
    const int tid = threadIdx.x;
    const int64_t per = (m + nblk - 1) / nblk;
    const int64_t lo = blk * per;
    const int64_t hi = (lo + per < m) ? lo + per : m;
    for (int e = tid; e < n * k; e += 256) Xs[e] = X[(e % n) + (int64_t)(e / n) * ldx];
    for (int e = tid; e < kResRows * k; e += 256) {
        Ss[e] = 0.0;
        Fs[e] = 0.0;
    }
    // accumulators of A^T Rr: thread owns (j, c) pairs e = tid + 256 q
    constexpr int kMaxOwn = 8;              // n * k <= 2048
    double acc[kMaxOwn];
#pragma unroll
    for (int q = 0; q < kMaxOwn; ++q) acc[q] = 0.0;
    for (int64_t r0 = lo; r0 < hi; r0 += kResRows) {
        const int rows = (int)((hi - r0 < kResRows) ? hi - r0 : kResRows);
        __syncthreads();
        for (int e = tid; e < kResRows * n; e += 256) {
            const int r = e % kResRows, j = e / kResRows;
            At[r * n + j] = (r < rows) ? A[r0 + r + (int64_t)j * lda] : 0.0;
        }
        for (int e = tid; e < kResRows * k; e += 256) {
            const int r = e % kResRows, c = e / kResRows;
            Rt[r * k + c] = (r < rows) ? Rr[r0 + r + (int64_t)c * m] : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < kResRows * k; e += 256) {
            const int r = e % kResRows, c = e / kResRows;
            if (r >= rows) continue;
            double s = B[r0 + r + (int64_t)c * ldb];
            for (int j = 0; j < n; ++j) s = fma(-At[r * n + j], Xs[j + n * c], s);
            Ss[r * k + c] = fma(s, s, Ss[r * k + c]);
            const double fv = s - Rt[r * k + c];
            Fs[r * k + c] = fma(fv, fv, Fs[r * k + c]);
            F[r0 + r + (int64_t)c * m] = fv;
        }
#pragma unroll
        for (int q = 0; q < kMaxOwn; ++q) {
            const int e = tid + 256 * q;
            if (e < n * k) {
                const int j = e % n, c = e / n;
                double s = acc[q];
                for (int r = 0; r < rows; ++r) s = fma(At[r * n + j], Rt[r * k + c], s);
                acc[q] = s;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxOwn; ++q) {
        const int e = tid + 256 * q;
        if (e < n * k) gpart[blk * n * k + e] = acc[q];
    }
    __syncthreads();
    if (tid < k) {
        double s = 0.0, f = 0.0;
        for (int r = 0; r < kResRows; ++r) {
            s += Ss[r * k + tid];
            f += Fs[r * k + tid];
        }
        rpart[blk * 2 * k + tid] = s;
        rpart[blk * 2 * k + k + tid] = f;
    }
}

// Sum over the 16 lanes of a row (lane bits 0..3), the same bits in all 16.
__device__ __forceinline__ double row16_sum(double v) {
    v = sum_quad(v);
    v += __shfl_xor(v, 4);
    v += dpp_f64<kDppRowRor8>(v);
    return v;
}

// Rows p[0 .. nv) of one column (zeros elsewhere, all zeros if !ok): two
// 16-byte loads when all four rows are there and p is 16-byte aligned.
__device__ __forceinline__ void load_rows4(const double *__restrict__ p, bool ok, int nv, bool al,
                                           double (&v)[4]) {
    if (ok && nv == 4 && al) {
        const double2 x0 = reinterpret_cast<const double2 *>(p)[0];
        const double2 x1 = reinterpret_cast<const double2 *>(p)[1];
        v[0] = x0.x; v[1] = x0.y; v[2] = x1.x; v[3] = x1.y;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (ok && q < nv) ? p[q] : 0.0;
    }
}

// The same pass as resid_block for n <= 16 MAXJT columns and k <= K
// right-hand sides, laid out for HBM: lane = 16 rg + cg takes column
// 16 jt + cg of the 16-column tile jt and the 4 consecutive rows 4 rg .. 4 rg + 3
// of a 16-row block (16-byte loads), so an instruction reads whole lines.
// A^T Rr accumulates per lane (one column, many rows) and is summed over
// the lanes once at the end; A X is summed over the 16 column lanes of a
// row per block.  Blocks of rows are multiples of 16; block blk covers
// rows [blk per, (blk + 1) per) (possibly empty).
template <int MAXJT, int K>
__device__ __forceinline__ void resid_fast(const double *__restrict__ A, int64_t lda, int64_t m, int n,
                                           const double *__restrict__ B, int64_t ldb,
                                           const double *__restrict__ X, int64_t ldx,
                                           const double *__restrict__ Rr, double *__restrict__ F, int k,
                                           double *__restrict__ gpart, double *__restrict__ rpart,
                                           int64_t blk, int64_t nblk) {
    __shared__ double gsh[4][MAXJT * 16 * K];
    __shared__ double ssh[4][K];
    __shared__ double fsh[4][K];
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int njt = (n + 15) >> 4;
    const int64_t per = ((m + nblk - 1) / nblk + 15) / 16 * 16;
    const int64_t lo = blk * per;
    const int64_t hi = (lo + per < m) ? lo + per : m;
    const bool al = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 1) == 0;
    double xr[MAXJT][K], g[MAXJT][K];
#pragma unroll
    for (int jt = 0; jt < MAXJT; ++jt)
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const int col = 16 * jt + l16;
            xr[jt][c] = (jt < njt && col < n && c < k) ? X[col + (int64_t)c * ldx] : 0.0;
            g[jt][c] = 0.0;
        }
    double ss = 0.0;   // squared (B - A X) of column l16 (lanes l16 < k)
    double ff = 0.0;   // squared F of column l16
    for (int64_t rb0 = lo + 16 * w; rb0 < hi; rb0 += 64) {
        const int64_t rb = rb0 + 4 * l4;
        const int nv = (int)((hi - rb >= 4) ? 4 : (hi - rb > 0 ? hi - rb : 0));
        double rr[4][K], sx[4][K];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < K; ++c) {
                rr[q][c] = (q < nv && c < k) ? Rr[rb + q + (int64_t)c * m] : 0.0;
                sx[q][c] = 0.0;
            }
#pragma unroll
        for (int jt = 0; jt < MAXJT; ++jt) {
            if (jt < njt) {   // a guard, not a break: the loop must unroll fully
                const int col = 16 * jt + l16;
                double a4[4];
                load_rows4(A + rb + (int64_t)col * lda, col < n, nv, al, a4);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        sx[q][c] = fma(a4[q], xr[jt][c], sx[q][c]);
                        g[jt][c] = fma(a4[q], rr[q][c], g[jt][c]);
                    }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < K; ++c) sx[q][c] = row16_sum(sx[q][c]);
        if (l16 < k) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= nv) continue;
                double ax = sx[q][0], rc = rr[q][0];
#pragma unroll
                for (int c = 1; c < K; ++c) {
                    ax = (l16 == c) ? sx[q][c] : ax;
                    rc = (l16 == c) ? rr[q][c] : rc;
                }
                const int64_t row = rb + q;
                const double sres = B[row + (int64_t)l16 * ldb] - ax;
                ss = fma(sres, sres, ss);
                const double fv = sres - rc;
                ff = fma(fv, fv, ff);
                F[row + (int64_t)l16 * m] = fv;
            }
        }
    }
    // totals over the 4 row groups of a wave, then over the waves in order
#pragma unroll
    for (int jt = 0; jt < MAXJT; ++jt)
#pragma unroll
        for (int c = 0; c < K; ++c) g[jt][c] = pair_sum32(pair_sum16(g[jt][c]));
    ss = pair_sum32(pair_sum16(ss));
    ff = pair_sum32(pair_sum16(ff));
    if (l4 == 0) {
#pragma unroll
        for (int jt = 0; jt < MAXJT; ++jt)
#pragma unroll
            for (int c = 0; c < K; ++c) gsh[w][(16 * jt + l16) * K + c] = g[jt][c];
        if (l16 < K) {
            ssh[w][l16] = ss;
            fsh[w][l16] = ff;
        }
    }
    __syncthreads();
    for (int e = tid; e < n * k; e += 256) {
        const int j = e % n, c = e / n, idx = j * K + c;
        gpart[blk * n * k + e] = ((gsh[0][idx] + gsh[1][idx]) + gsh[2][idx]) + gsh[3][idx];
    }
    if (tid < k) {
        rpart[blk * 2 * k + tid] = ((ssh[0][tid] + ssh[1][tid]) + ssh[2][tid]) + ssh[3][tid];
        rpart[blk * 2 * k + k + tid] = ((fsh[0][tid] + fsh[1][tid]) + fsh[2][tid]) + fsh[3][tid];
    }
}

template <int MAXJT, int K>
__global__ __launch_bounds__(256) void k_lsq_resid_fast(const double *__restrict__ A, int64_t lda, int64_t m,
                                                        int n, const double *__restrict__ B, int64_t ldb,
                                                        const double *__restrict__ X, int64_t ldx,
                                                        const double *__restrict__ Rr, double *__restrict__ F,
                                                        int k, double *__restrict__ gpart,
                                                        double *__restrict__ rpart) {
    resid_fast<MAXJT, K>(A, lda, m, n, B, ldb, X, ldx, Rr, F, k, gpart, rpart, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_lsq_resid(const double *__restrict__ A, int64_t lda, int64_t m,
                                                   int n, const double *__restrict__ B, int64_t ldb,
                                                   const double *__restrict__ X, int64_t ldx,
                                                   const double *__restrict__ Rr, double *__restrict__ F,
                                                   int k, double *__restrict__ gpart,
                                                   double *__restrict__ rpart) {
    extern __shared__ double sh[];
    resid_block(A, lda, m, n, B, ldb, X, ldx, Rr, F, k, gpart, rpart, blockIdx.x, gridDim.x, sh);
}

// One workgroup: g = -sum_b gpart[b];  R^T h = g;  dx = R^{-1} (d_1 - h)
// with d_1 = F[0:n] (= (Q^T f)[0:n] on entry);  X += dx;  F[0:n] = h.
// status[0] = sweeps done, status[1] = 1 when converged or stalled,
// hist[c] = ||dx_c|| / ||x_c|| of the last sweep and, if gnorm is set,
// gnorm[c] = ||g_c||.  A sweep counts as final when every column either
// converged or stalled (its correction shrank by less than 10 %).  A column
// has converged when the error left after this sweep's correction,
// estimated as rho ||dx|| with rho = ||dx|| / ||dx_prev|| the observed
// contraction of the iteration (at most 1), is below tol ||x|| -- so a
// sweep whose correction is already far below the tolerance is not needed
// just to confirm it.
__device__ __forceinline__ void refine_step(const double *__restrict__ R, int n, double *__restrict__ F,
                                            int64_t m, int k, const double *__restrict__ gpart, int nblocks,
                                            double *__restrict__ X, int64_t ldx, double tol,
                                            int32_t *__restrict__ status, double *__restrict__ hist,
                                            double *__restrict__ gnorm) {
    __shared__ double g[256];
    const int tid = threadIdx.x, lane = tid & 63;
    bool all_ok = true;
    for (int c = 0; c < k; ++c) {
        // g = -sum_b gpart[b] (every thread), in a fixed order per entry:
        // even blocks into s0, odd blocks into s1, in block order.  The loads
        // go out 16 at a time ahead of the adds (the sum waits on memory
        // latency, not on the adds); the order of the adds is unchanged.
        __syncthreads();
        for (int j = tid; j < n; j += blockDim.x) {
            double s0 = 0.0, s1 = 0.0;
            if (gpart) {
                const double *__restrict__ p = gpart + j + (int64_t)n * c;
                const int64_t bs = (int64_t)n * k;
                int b = 0;
                for (; b + 15 < nblocks; b += 16) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) v[u] = p[(int64_t)(b + u) * bs];
#pragma unroll
                    for (int u = 0; u < 16; u += 2) {
                        s0 += v[u];
                        s1 += v[u + 1];
                    }
                }
                for (; b + 1 < nblocks; b += 2) {
                    s0 += p[(int64_t)b * bs];
                    s1 += p[(int64_t)(b + 1) * bs];
                }
                if (b < nblocks) s0 += p[(int64_t)b * bs];
            }
            g[j] = -(s0 + s1);
        }
        __syncthreads();
        if (tid < 64) {   // the solves run on one wave
            double h[4], dx[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane + 64 * q;
                h[q] = (i < n) ? g[i] : 0.0;
            }
            if (gnorm) {
                double gg = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) gg = fma(h[q], h[q], gg);
                gg = wave_sum(gg);
                if (lane == 0) gnorm[c] = sqrt(gg);
            }
            wave_fwdsub_t(R, n, h);                       // R^T h = g
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane + 64 * q;
                dx[q] = (i < n) ? F[i + m * c] - h[q] : 0.0;
            }
            wave_backsub(R, n, dx);                       // R dx = d_1 - h
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane + 64 * q;
                if (i < n) {
                    const double xn = X[i + ldx * c] + dx[q];
                    a = fma(dx[q], dx[q], a);
                    b = fma(xn, xn, b);
                    X[i + ldx * c] = xn;
                    F[i + m * c] = h[q];
                }
            }
            a = wave_sum(a);
            b = wave_sum(b);
            const double rel = sqrt(a) / fmax(sqrt(b), 1e-300);
            const double prev = hist[c];
            const double rho = (status[0] >= 1 && prev > 0.0) ? fmin(rel / prev, 1.0) : 1.0;
            const bool done = (rho * rel <= tol) || (status[0] >= 1 && rel > 0.9 * prev) || !(rel == rel);
            all_ok = all_ok && done;
            if (lane == 0) hist[c] = rel;
        }
    }
    if (tid == 0) {
        status[0] += 1;
        status[1] = all_ok ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_lsq_refine(const double *__restrict__ R, int n,
                                                    double *__restrict__ F, int64_t m, int k,
                                                    const double *__restrict__ gpart, int nblocks,
                                                    double *__restrict__ X, int64_t ldx, double tol,
                                                    int32_t *__restrict__ status,
                                                    double *__restrict__ hist, double *__restrict__ gnorm) {
    refine_step(R, n, F, m, k, gpart, nblocks, X, ldx, tol, status, hist, gnorm);
}

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, int64_t count) {
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < count;
         e += (int64_t)blockDim.x * gridDim.x)
        y[e] += x[e];
}

__global__ void k_status_init(int32_t *status, double *hist, int k) {
    if (threadIdx.x == 0) {
        status[0] = 0;
        status[1] = 0;
    }
    if ((int)threadIdx.x < k) hist[threadIdx.x] = 1.0;
}

// Upper bound on the least-squares backward error of x (Sec. 1 of the
// paper only names least squares; the bound is the normwise one used to
// judge refinement):  with the last residual pass's s = b - A x,
// f = b - r - A x and g = -A^T r,
//     ||A^T s|| <= ||g|| + ||A|| ||f||,
//     eta = ||A^T s|| / (||A|| (||A|| ||x|| + ||s||)),
// and ||A||_F = ||R||_F (A = QR, Q orthogonal).
__device__ __forceinline__ double eta_bound(double gn, double fn, double sn, double xn, double an) {
    const double den = an * fma(an, xn, sn);
    return den > 0.0 ? fma(an, fn, gn) / den : 0.0;
}

constexpr double kEtaMax = 1e-12;   // a refined x above this bound is flagged (dinfo = -3)

// ||R||_F of the n x n triangle, by one workgroup (every thread returns it).
__device__ __forceinline__ double tri_fnorm(const double *__restrict__ R, int n, double *red) {
    double s = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        if (r <= c) s = fma(R[e], R[e], s);
    }
    s = wave_sum(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return sqrt(t);
}

// Last step of a refined solve: info from the diagonal of R (LAPACK dtrtrs
// convention: X untouched when R_jj == 0), X = Xw otherwise, residual norms
// ||b_c - A x_c|| and the backward-error bound eta_c (eta_out) from the last
// residual pass; info = -2 for a non-finite residual, -3 when some eta_c
// exceeds kEtaMax (the refinement stalled or ran out of sweeps before x was
// FP64-accurate).
__global__ __launch_bounds__(256) void k_mixed_final(const double *R, int n, int k, const double *Xw,
                                                     double *X, int64_t ldx, double *resid, int32_t *dinfo,
                                                     int merge, const double *rpart, int nblocks,
                                                     const double *gnorm, double *eta_out) {
    __shared__ int info;
    __shared__ double red[4];
    const int tid = threadIdx.x;
    if (tid == 0) {
        info = 0;
        for (int j = 0; j < n; ++j)
            if (R[j + j * n] == 0.0) {
                info = j + 1;
                break;
            }
    }
    const double an = tri_fnorm(R, n, red);
    __syncthreads();
    bool bad = false, loose = false;
    if (tid < k) {
        double s = 0.0, f = 0.0, xx = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            s += rpart[(int64_t)b * 2 * k + tid];
            f += rpart[(int64_t)b * 2 * k + k + tid];
        }
        for (int j = 0; j < n; ++j) xx = fma(Xw[j + n * tid], Xw[j + n * tid], xx);
        const double rn = sqrt(s);
        const double eta = eta_bound(gnorm[tid], sqrt(f), rn, sqrt(xx), an);
        if (resid) resid[tid] = rn;
        if (eta_out) eta_out[tid] = eta;
        bad = !(rn - rn == 0.0);
        loose = !(eta <= kEtaMax);
    }
    const int anybad = __syncthreads_or(bad);
    const int anyloose = __syncthreads_or(loose);
    // merge: a later group of right-hand sides keeps an earlier nonzero code
    if (tid == 0 && dinfo && !(merge && *dinfo != 0))
        *dinfo = info ? info : (anybad ? -2 : (anyloose ? -3 : 0));
    if (info) return;
    for (int e = tid; e < n * k; e += 256) X[(e % n) + (int64_t)(e / n) * ldx] = Xw[e];
}

hipError_t launch_mixed_final(const double *R, int n, int k, const double *Xw, double *X, int64_t ldx,
                              double *resid, int32_t *dinfo, int merge, const double *rpart, int nblocks,
                              const double *gnorm, double *eta_out, hipStream_t st) {
    ProfScope ps("lsq_final", st);
    hipLaunchKernelGGL(k_mixed_final, dim3(1), dim3(256), 0, st, R, n, k, Xw, X, ldx, resid, dinfo, merge,
                       rpart, nblocks, gnorm, eta_out);
    return hipGetLastError();
}

// ---- batched refinement (one right-hand side per matrix) ----

// F = b, Rr = 0, x = 0, flags cleared.
__global__ void k_lsq_init_b(const BMat *__restrict__ mats, const int *__restrict__ list) {
    const BMat &M = mats[list[blockIdx.y]];
    const int64_t m = M.pa.m;
    for (int64_t r = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; r < m;
         r += (int64_t)blockDim.x * gridDim.x) {
        M.F[r] = M.b[r];
        if (M.prec) M.Rr[r] = 0.0;
    }
    if (blockIdx.x == 0) {
        for (int j = threadIdx.x; j < M.pa.n; j += blockDim.x) M.Xw[j] = 0.0;
        if (threadIdx.x == 0) {
            M.status[0] = 0;
            M.status[1] = 0;
            M.hist[0] = 1.0;
            M.hist[1] = 0.0;
            M.hist[2] = 0.0;
        }
    }
}

__global__ __launch_bounds__(256) void k_resid_b(const BMat *__restrict__ mats, const int *__restrict__ list,
                                                 int sweep) {
    extern __shared__ double sh[];
    const BMat &M = mats[list[blockIdx.y]];
    if ((int)blockIdx.x >= M.nb) return;
    if (sweep > 0 && M.status[1]) return;
    if (M.pa.n <= 64)
        resid_fast<4, 1>(M.A, M.lda, M.pa.m, M.pa.n, M.b, M.pa.m, M.Xw, M.pa.n, M.Rr, M.F, 1, M.gpart, M.rpart,
                         blockIdx.x, M.nb);
    else
        resid_block(M.A, M.lda, M.pa.m, M.pa.n, M.b, M.pa.m, M.Xw, M.pa.n, M.Rr, M.F, 1, M.gpart, M.rpart,
                    blockIdx.x, M.nb, sh);
}

// One workgroup per matrix.  Sweep 0 is the plain solve (g = 0); an FP64
// matrix stops there, with ||(Q^T b)[n:m]|| as its residual norm.
__global__ __launch_bounds__(256) void k_refine_b(const BMat *__restrict__ mats, const int *__restrict__ list,
                                                  int sweep, double tol) {
    __shared__ double red[256];
    const BMat &M = mats[list[blockIdx.x]];
    if (sweep > 0 && M.status[1]) return;
    const int n = M.pa.n;
    const int64_t m = M.pa.m;
    if (!M.prec) {
        double s = 0.0;
        for (int64_t r = n + threadIdx.x; r < m; r += 256) s = fma(M.F[r], M.F[r], s);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) M.hist[1] = sqrt(red[0]);
        __syncthreads();
    }
    refine_step(M.R, n, M.F, m, 1, sweep > 0 ? M.gpart : nullptr, M.nb, M.Xw, n, tol, M.status, M.hist,
                M.prec ? M.hist + 2 : nullptr);
    if (!M.prec && threadIdx.x == 0) M.status[1] = 1;
}

__global__ void k_axpy_b(const BMat *__restrict__ mats, const int *__restrict__ list, int sweep) {
    const BMat &M = mats[list[blockIdx.y]];
    if (sweep > 0 && M.status[1]) return;
    for (int64_t r = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; r < M.pa.m;
         r += (int64_t)blockDim.x * gridDim.x)
        M.Rr[r] += M.F[r];
}

// Per matrix: info, residual norm and x; a mixed matrix also gets the
// backward-error bound of k_mixed_final (info = -3 above kEtaMax).
__global__ void k_final_b(const BMat *__restrict__ mats, const int *__restrict__ list) {
    __shared__ int info;
    __shared__ double red[4];
    const BMat &M = mats[list[blockIdx.x]];
    const int n = M.pa.n;
    if (threadIdx.x == 0) {
        info = 0;
        for (int j = 0; j < n; ++j)
            if (M.R[j + j * n] == 0.0) {
                info = j + 1;
                break;
            }
    }
    const double an = M.prec ? tri_fnorm(M.R, n, red) : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double rn;
        bool loose = false;
        if (M.prec) {
            double s = 0.0, f = 0.0, xx = 0.0;
            for (int b = 0; b < M.nb; ++b) {
                s += M.rpart[2 * b];
                f += M.rpart[2 * b + 1];
            }
            for (int j = 0; j < n; ++j) xx = fma(M.Xw[j], M.Xw[j], xx);
            rn = sqrt(s);
            loose = !(eta_bound(M.hist[2], sqrt(f), rn, sqrt(xx), an) <= kEtaMax);
        } else {
            rn = M.hist[1];
        }
        *M.resid = rn;
        *M.info = info ? info : (!(rn - rn == 0.0) ? -2 : (loose ? -3 : 0));
    }
    __syncthreads();
    if (info) return;
    for (int j = threadIdx.x; j < n; j += blockDim.x) M.x[j] = M.Xw[j];
}

static unsigned rows_grid(int64_t gx) { return (unsigned)(gx < 1 ? 1 : (gx > 1024 ? 1024 : gx)); }

hipError_t launch_lsq_init_b(const BMat *mats, const int *list, int cnt, int64_t gx, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    ProfScope ps("batch_lsq_init", st);
    hipLaunchKernelGGL(k_lsq_init_b, dim3(rows_grid(gx), (unsigned)cnt), dim3(256), 0, st, mats, list);
    return hipGetLastError();
}

hipError_t launch_resid_b(const BMat *mats, const int *list, int cnt, int64_t gx, int sweep, hipStream_t st) {
    if (cnt <= 0 || gx <= 0) return hipSuccess;
    // n <= 64, k = 1
    const size_t sh = sizeof(double) * ((size_t)kResRows * 64 + 64 + 3 * (size_t)kResRows);
    ProfScope ps("batch_lsq_resid", st);
    hipLaunchKernelGGL(k_resid_b, dim3((unsigned)gx, (unsigned)cnt), dim3(256), sh, st, mats, list, sweep);
    return hipGetLastError();
}

hipError_t launch_refine_b(const BMat *mats, const int *list, int cnt, int sweep, double tol, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    ProfScope ps("batch_lsq_refine", st);
    hipLaunchKernelGGL(k_refine_b, dim3((unsigned)cnt), dim3(256), 0, st, mats, list, sweep, tol);
    return hipGetLastError();
}

hipError_t launch_axpy_b(const BMat *mats, const int *list, int cnt, int64_t gx, int sweep, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    ProfScope ps("batch_axpy", st);
    hipLaunchKernelGGL(k_axpy_b, dim3(rows_grid(gx), (unsigned)cnt), dim3(256), 0, st, mats, list, sweep);
    return hipGetLastError();
}

hipError_t launch_final_b(const BMat *mats, const int *list, int cnt, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    ProfScope ps("batch_lsq_final", st);
    hipLaunchKernelGGL(k_final_b, dim3((unsigned)cnt), dim3(256), 0, st, mats, list);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                         int64_t cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    ProfScope ps("to_f32", st);
    hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

// At most 768 workgroups: the widest line-wide residual pass (16 accumulator
// pairs per lane, 152 VGPRs) keeps three 256-thread workgroups on each of the
// 256 CUs, so a tall matrix's whole pass is resident at once instead of
// leaving a partly filled second dispatch wave.
int resid_blocks(int64_t m) {
    constexpr int64_t kResident = 3 * 256;
    static_assert(kResident <= kRefineBlocks, "partials buffer");
    int64_t b = (m + 2047) / 2048;
    return (int)(b < 1 ? 1 : (b > kResident ? kResident : b));
}

hipError_t launch_lsq_resid(const double *A, int64_t lda, int64_t m, int n, const double *B, int64_t ldb,
                            const double *X, int64_t ldx, const double *Rr, double *F, int k,
                            double *gpart, double *rpart, int nblocks, hipStream_t st) {
    // the line-wide pass for up to 16 MAXJT columns x K right-hand sides
    // (MAXJT K <= 32 accumulators per lane), the tiled pass otherwise
    const int njt = (n + 15) / 16;
    const int jt = njt <= 4 ? 4 : (njt <= 8 ? 8 : (njt <= 16 ? 16 : 0));
    const int kk = k <= 1 ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : (k <= 8 ? 8 : 0)));
    if (jt > 0 && kk > 0 && jt * kk <= 32) {
        ProfScope ps("lsq_resid", st);
#define TSQR_RESID_FAST(J, KK)                                                                              \
    if (jt == J && kk == KK) {                                                                          \
        hipLaunchKernelGGL((k_lsq_resid_fast<J, KK>), dim3(nblocks), dim3(256), 0, st, A, lda, m, n, B, ldb, \
                           X, ldx, Rr, F, k, gpart, rpart);                                             \
        return hipGetLastError();                                                                       \
    }
        TSQR_RESID_FAST(4, 1) TSQR_RESID_FAST(4, 2) TSQR_RESID_FAST(4, 4) TSQR_RESID_FAST(4, 8)
        TSQR_RESID_FAST(8, 1) TSQR_RESID_FAST(8, 2) TSQR_RESID_FAST(8, 4)
        TSQR_RESID_FAST(16, 1) TSQR_RESID_FAST(16, 2)
#undef TSQR_RESID_FAST
    }
    const size_t sh =
        sizeof(double) * ((size_t)kResRows * n + (size_t)n * k + 3 * (size_t)kResRows * k);
    hipError_t e = hipFuncSetAttribute((const void *)k_lsq_resid,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("lsq_resid", st);
    hipLaunchKernelGGL(k_lsq_resid, dim3(nblocks), dim3(256), sh, st, A, lda, m, n, B, ldb, X, ldx, Rr, F,
                       k, gpart, rpart);
    return hipGetLastError();
}

hipError_t launch_lsq_refine(const double *R, int n, double *F, int64_t m, int k, const double *gpart,
                             int nblocks, double *X, int64_t ldx, double tol, int32_t *status,
                             double *hist, double *gnorm, hipStream_t st) {
    ProfScope ps("lsq_refine", st);
    hipLaunchKernelGGL(k_lsq_refine, dim3(1), dim3(256), 0, st, R, n, F, m, k, gpart, nblocks, X, ldx, tol,
                       status, hist, gnorm);
    return hipGetLastError();
}

hipError_t launch_axpy(double *y, const double *x, int64_t count, hipStream_t st) {
    ProfScope ps("axpy", st);
    hipLaunchKernelGGL(k_axpy, dim3(2048), dim3(256), 0, st, y, x, count);
    return hipGetLastError();
}

hipError_t launch_status_init(int32_t *status, double *hist, int k, hipStream_t st) {
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, st, status, hist, k);
    return hipGetLastError();
}

}  // namespace tsqr
