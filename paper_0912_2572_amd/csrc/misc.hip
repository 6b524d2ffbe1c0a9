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

// One wave per right-hand side: info from the diagonal of R, the residual
// norm from the partials, then X = R^{-1} C[0:n] by back substitution.
__global__ __launch_bounds__(64) void k_lsq_final(const double *R, int n, const double *C, int64_t ldc,
                                                  int64_t k, double *X, int64_t ldx, double *resid,
                                                  int32_t *dinfo, const double *partial, int nparts) {
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    // the right-hand side and the residual partials are loaded before the
    // diagonal test, so the three groups of loads overlap
    double xr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
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
    wave_backsub(R, n, xr);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i < n) X[i + c * ldx] = xr[q];
    }
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

hipError_t launch_lsq_finish(const double *R, int n, const double *C, int64_t ldc, int64_t m, int64_t k,
                             double *X, int64_t ldx, double *resid, int32_t *dinfo, double *partial,
                             hipStream_t st) {
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
    hipLaunchKernelGGL(k_lsq_final, dim3((unsigned)k), dim3(64), 0, st, R, n, C, ldc, k, X, ldx, resid, dinfo,
                       partial, blocks);
    return hipGetLastError();
}

}  // namespace tsqr
