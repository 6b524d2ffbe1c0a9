// misc.hip -- small kernels around the TSQR core: the [D; 0] seed of the
// thin Q, 2-D copies, and the last steps of least squares (back substitution
// with R and the residual norms ||(Q^T B)[n:m, j]||_2).
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace tsqr {

// Q (m x n) = [D; 0], D = diag(d): the thin Q is Q_full [D; 0] (R <- D R,
// Q <- Q D makes the factorization unique, Sec. 2.2).
__global__ void k_fill_identity_signs(double *Q, int64_t ldq, int64_t m, int n, const double *d) {
    const int64_t total = m * (int64_t)n;
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < total;
         e += (int64_t)blockDim.x * gridDim.x) {
        const int64_t r = e % m, c = e / m;
        Q[r + c * ldq] = (r == c) ? d[c] : 0.0;
    }
}

__global__ void k_fill(double *p, int64_t count, double value) {
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < count;
         e += (int64_t)blockDim.x * gridDim.x)
        p[e] = value;
}

__global__ void k_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                       int64_t cols) {
    const int64_t total = rows * cols;
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < total;
         e += (int64_t)blockDim.x * gridDim.x) {
        const int64_t r = e % rows, c = e / rows;
        dst[r + c * ldd] = src[r + c * lds];
    }
}

constexpr int kResidBlocks = 512;

// partial[b][c] = sum of C[r][c]^2 over the rows n..m-1 owned by block b
// (contiguous row ranges, fixed summation order).
__global__ __launch_bounds__(256) void k_resid_partial(const double *C, int64_t ldc, int64_t m, int n,
                                                       int64_t k, double *partial, int32_t *dinfo) {
    __shared__ double red[256];
    // the info word the final kernel raises with atomics starts at zero
    if (dinfo && blockIdx.x == 0 && threadIdx.x == 0) *dinfo = 0;
    const int64_t rows = m - n;
    const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t lo = n + (int64_t)blockIdx.x * per;
    const int64_t hi = (lo + per < m) ? lo + per : m;
    for (int64_t c = 0; c < k; ++c) {
        double s = 0.0;
        for (int64_t r = lo + threadIdx.x; r < hi; r += 256) {
            const double v = C[r + c * ldc];
            s = fma(v, v, s);
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x * k + c] = red[0];
        __syncthreads();
    }
}

// Back substitution R x = b for 256 < n <= 64 Q (lane l holds entries
// l + 64 q, q < Q): the one-wave scheme of wave_backsub with Q slots per lane.
template <int Q>
__device__ __forceinline__ double pick_slot(const double (&xr)[Q], int q) {
    double v = xr[0];
#pragma unroll
    for (int u = 1; u < Q; ++u) v = (q == u) ? xr[u] : v;
    return v;
}

template <int Q>
__device__ __forceinline__ void wide_backsub(const double *__restrict__ R, int n, double (&xr)[Q]) {
    const int lane = threadIdx.x & 63;
    constexpr int D = kSolveAhead;
    double col[D][Q], dg[D];
    auto fetch = [&](int j, double (&cc)[Q], double &d) {
        const int jj = j < 0 ? 0 : j;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = lane + 64 * q;
            const double v = R[(i < jj ? i : 0) + (int64_t)jj * n];
            cc[q] = (i < jj) ? v : 0.0;
        }
        d = R[jj + (int64_t)jj * n];
    };
    auto step = [&](int j, const double (&cc)[Q], double d) {
        const int qj = j >> 6, lj = j & 63;
        const double xj = wave_bcast(pick_slot<Q>(xr, qj), lj) / d;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            xr[q] = fma(-cc[q], xj, xr[q]);
            if (q == qj && lane == lj) xr[q] = xj;
        }
    };
#pragma unroll
    for (int u = 0; u < D; ++u) fetch(n - 1 - u, col[u], dg[u]);
    int j0 = n - 1;
    for (; j0 - (D - 1) >= 0; j0 -= D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            step(j0 - u, col[u], dg[u]);
            fetch(j0 - u - D, col[u], dg[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < D - 1; ++u)
        if (j0 - u >= 0) step(j0 - u, col[u], dg[u]);
}

// One wave per right-hand side: info from the diagonal of R, the residual
// norm from the partials, then X = R^{-1} C[0:n] by back substitution
// (Q = 4 slots per lane for n <= 256, 16 for n <= 1024).
template <int Q>
__global__ __launch_bounds__(64) void k_lsq_final(const double *R, int n, const double *C, int64_t ldc,
                                                  int64_t k, double *X, int64_t ldx, double *resid,
                                                  int32_t *dinfo, const double *partial, int nparts) {
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    // the right-hand side and the residual partials are loaded before the
    // diagonal test, so the three groups of loads overlap
    double xr[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = lane + 64 * q;
        xr[q] = (i < n) ? C[i + c * ldc] : 0.0;
    }
    double s = 0.0;
    for (int b = lane; b < nparts; b += 64) s += partial[(int64_t)b * k + c];
    int info = 0;
    for (int j0 = 0; j0 < n && !info; j0 += 64) {
        const int j = j0 + lane;
        const bool zero = j < n && R[j + (int64_t)j * n] == 0.0;
        const unsigned long long mask = __ballot(zero);
        if (mask) info = j0 + __ffsll((long long)mask);
    }
    const double rn = sqrt(wave_sum(s));
    if (lane == 0) {
        if (resid) resid[c] = rn;
        // the lowest code over the columns: info first, then -2
        if (dinfo) {
            const int32_t code = info ? info : (!(rn - rn == 0.0) ? -2 : 0);
            if (code > 0) atomicMax(dinfo, code);   // info is the same for every column
            else if (code < 0) atomicMin(dinfo, code);
        }
    }
    if (info) return;
    if constexpr (Q == 4) wave_backsub(R, n, xr);
    else wide_backsub<Q>(R, n, xr);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = lane + 64 * q;
        if (i < n) X[i + c * ldx] = xr[q];
    }
}

// Largest value over the 64 lanes, identical in every lane.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) v = fmax(v, __shfl_xor(v, s));
    return v;
}

// Index (< n) of the entry of largest magnitude of the wave's vector (lane l
// holds entries l + 64 q in x[q]); ties go to the lower index.  Identical in
// every lane.
__device__ __forceinline__ int wave_argmax_abs(const double (&x)[4], int n) {
    const int lane = threadIdx.x & 63;
    double best = -1.0;
    int bi = n;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        const double a = fabs(x[q]);
        if (i < n && a > best) {
            best = a;
            bi = i;
        }
    }
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const double ob = __shfl_xor(best, s);
        const int oi = __shfl_xor(bi, s);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    return bi;
}

// The 1-norm condition estimate of R: ||R||_1 times a lower bound on
// ||R^{-1}||_1 by Hager's method (1984) with Higham's refinements (1988):
// y = R^{-1} (e / n); then up to four times: xi = sgn(y), z = R^{-T} xi,
// j = argmax |z_j|, y = R^{-1} e_j, stopping when the sign vector repeats,
// the estimate ||y||_1 stops growing (the larger of the last two is kept) or
// the argmax repeats; finally the alternating vector x_i = (-1)^i (1 + i /
// (n - 1)) gives the bound 2 ||R^{-1} x||_1 / (3n) when that is larger.
// sgn(0) = +1.  One wave, no barrier; the solves are the one-wave ones.
__global__ __launch_bounds__(64) void k_cond_est(const double *R, int n, double *kappa) {
    const int lane = threadIdx.x;
    double cmax = 0.0;
    bool zero = false;
    for (int q = 0; q < 4; ++q) {
        const int j = lane + 64 * q;
        if (j < n) {
            double s = 0.0;
            for (int i = 0; i <= j; ++i) s += fabs(R[i + (int64_t)j * n]);
            cmax = fmax(cmax, s);
            zero = zero || R[j + (int64_t)j * n] == 0.0;
        }
    }
    const double norm = wave_max(cmax);
    if (__ballot(zero)) {
        if (lane == 0) *kappa = INFINITY;
        return;
    }
    auto l1 = [&](const double (&v)[4]) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) s += fabs(v[q]);   // entries past n are zero
        return wave_sum(s);
    };
    double x[4], xi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = (lane + 64 * q < n) ? 1.0 / (double)n : 0.0;
    wave_backsub(R, n, x);
    double est;
    if (n == 1) {
        est = fabs(wave_bcast(x[0], 0));
    } else {
        est = l1(x);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xi[q] = (lane + 64 * q < n) ? (x[q] >= 0.0 ? 1.0 : -1.0) : 0.0;
            x[q] = xi[q];
        }
        wave_fwdsub_t(R, n, x);
        int j = wave_argmax_abs(x, n);
        for (int iter = 2; iter <= 5; ++iter) {
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = (lane + 64 * q == j) ? 1.0 : 0.0;
            wave_backsub(R, n, x);
            const double old = est;
            est = l1(x);
            bool diff = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (lane + 64 * q < n) {
                    const double sg = x[q] >= 0.0 ? 1.0 : -1.0;
                    diff = diff || sg != xi[q];
                    xi[q] = sg;
                }
            }
            if (!__ballot(diff) || est <= old) {
                est = fmax(est, old);
                break;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = xi[q];
            wave_fwdsub_t(R, n, x);
            const int jl = j;
            j = wave_argmax_abs(x, n);
            const double ajl = fabs(wave_bcast(pick4(x, jl >> 6), jl & 63));
            const double aj = fabs(wave_bcast(pick4(x, j >> 6), j & 63));
            if (ajl == aj) break;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = lane + 64 * q;
            x[q] = (i < n) ? ((i & 1) ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1)) : 0.0;
        }
        wave_backsub(R, n, x);
        const double t = 2.0 * l1(x) / (3.0 * (double)n);
        if (t > est) est = t;
    }
    if (lane == 0) *kappa = norm * est;
}

__global__ void k_info_clear(int32_t *dinfo) {
    if (threadIdx.x == 0) *dinfo = 0;
}

hipError_t launch_fill_identity_signs(double *Q, int64_t ldq, int64_t m, int n, const double *d,
                                      hipStream_t st) {
    ProfScope ps("fill_identity", st);
    hipLaunchKernelGGL(k_fill_identity_signs, dim3(2048), dim3(256), 0, st, Q, ldq, m, n, d);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t count, double value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    ProfScope ps("fill", st);
    unsigned blocks = (unsigned)((count + 255) / 256 < 2048 ? (count + 255) / 256 : 2048);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                       int64_t cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    ProfScope ps("copy", st);
    hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_cond_est(const double *R, int n, double *kappa, hipStream_t st) {
    if (n < 1 || n > 256) return hipErrorInvalidValue;
    ProfScope ps("cond_est", st);
    hipLaunchKernelGGL(k_cond_est, dim3(1), dim3(64), 0, st, R, n, kappa);
    return hipGetLastError();
}

hipError_t launch_lsq_finish(const double *R, int n, const double *C, int64_t ldc, int64_t m, int64_t k,
                             double *X, int64_t ldx, double *resid, int32_t *dinfo, double *partial,
                             hipStream_t st) {
    if (n < 1 || n > 1024) return hipErrorInvalidValue;
    int blocks = kResidBlocks;
    if (m - n < (int64_t)blocks * 256) blocks = (int)((m - n + 255) / 256);
    if (blocks < 1) blocks = 1;
    ProfScope ps("lsq_finish", st);
    if (m > n) {
        hipLaunchKernelGGL(k_resid_partial, dim3(blocks), dim3(256), 0, st, C, ldc, m, n, k, partial, dinfo);
    } else {
        blocks = 0;
        if (dinfo) hipLaunchKernelGGL(k_info_clear, dim3(1), dim3(64), 0, st, dinfo);
    }
    if (n > 256)
        hipLaunchKernelGGL(k_lsq_final<16>, dim3((unsigned)k), dim3(64), 0, st, R, n, C, ldc, k, X, ldx, resid,
                           dinfo, partial, blocks);
    else
        hipLaunchKernelGGL(k_lsq_final<4>, dim3((unsigned)k), dim3(64), 0, st, R, n, C, ldc, k, X, ldx, resid,
                           dinfo, partial, blocks);
    return hipGetLastError();
}

}  // namespace tsqr
