// orth.hip -- block orthogonalisation against an orthonormal basis, the
// step that block-iterative methods (block Krylov solvers, block
// eigensolvers) repeat to grow an orthogonal basis, with TSQR as the stable
// orthogonalisation of each new block (the paper's Scope section and
// Sec. 6: TSQR generates an orthogonal basis for a set of vectors stably,
// with few messages).
//
// For an orthonormal V (m x nv) and a new block W (m x b), two passes of
// block classical Gram-Schmidt
//     H1 = V^T W,  W <- W - V H1,  H2 = V^T W,  W <- W - V H2
// (the second pass restores orthogonality to V lost to rounding in the
// first), then TSQR of the projected W = Q R and Q written over W:
//     W_in = V (H1 + H2) + Q R,   [V Q]^T [V Q] = I.
//
// Kernels (FP64 matrix-core tiles v_mfma_f64_16x16x4f64, layout in mfma.h):
//   k_proj_partial  per row block, the nv x b partial V_blk^T W_blk: wave w
//                   owns 16 columns of a 64-column slice of V, a lane loads 4
//                   consecutive rows of one column (16-byte loads) and feeds
//                   4 matrix-core k-steps;
//   k_proj_reduce   H = sum of the partials in block order (deterministic);
//   k_proj_update   W -= V H: a wave owns 16 rows, the k-loop runs over V's
//                   columns 4 at a time; V is read in whole 128-byte row
//                   segments of a column.
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

namespace {

constexpr int kProjSlice = 64;   // V columns per workgroup of the partial pass

typedef double dv2o __attribute__((ext_vector_type(2)));

// Rows [r, r + 4) of column `col` (zeros past `hi` or past `cols`).
__device__ __forceinline__ void rows4(const double *__restrict__ M, int64_t ld, int64_t r, int64_t hi, int col,
                                      int cols, double (&v)[4]) {
    const bool ok = col < cols;
    const double *p = M + r + (int64_t)(ok ? col : 0) * ld;
    if (ok && r + 4 <= hi && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        const dv2o a = *reinterpret_cast<const dv2o *>(p);
        const dv2o b = *reinterpret_cast<const dv2o *>(p + 2);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (ok && r + q < hi) ? p[q] : 0.0;
    }
}

// Hpart[blk] (nv x b, column-major, ld nv) for columns [64 y, 64 y + 64)
// of V: block blk covers rows [blk per, (blk + 1) per), per a multiple of 16.
__global__ __launch_bounds__(256) void k_proj_partial(const double *__restrict__ V, int64_t ldv, int nv,
                                                      const double *__restrict__ W, int64_t ldw, int b,
                                                      int64_t m, int64_t per, double *__restrict__ Hpart) {
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int c0 = kProjSlice * blockIdx.y + 16 * w;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = (lo + per < m) ? lo + per : m;
    const int nJ = (b + 15) / 16;
    d4 acc[4];
#pragma unroll
    for (int J = 0; J < 4; ++J) acc[J] = d4_zero();
    if (c0 < nv) {
        for (int64_t r = lo; r < hi; r += 16) {
            // lane (i, kq) holds rows r + 4 kq .. r + 4 kq + 3; k-step s of
            // the tile uses row r + 4 kq + s for k-index kq
            const int64_t rr = r + 4 * kq;
            double a[4];
            rows4(V, ldv, rr, hi, c0 + i, nv, a);
#pragma unroll
            for (int J = 0; J < 4; ++J) {
                if (J < nJ) {
                    double bw[4];
                    rows4(W, ldw, rr, hi, 16 * J + i, b, bw);
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[J] = mfma_f64(a[s], bw[s], acc[J]);
                }
            }
        }
    }
    double *P = Hpart + (int64_t)blockIdx.x * nv * b;
#pragma unroll
    for (int J = 0; J < 4; ++J) {
        if (J >= nJ) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = c0 + d_row(q, lane), col = 16 * J + d_col(lane);
            if (row < nv && col < b) P[row + (int64_t)col * nv] = acc[J][q];
        }
    }
}

// H = sum over blocks of Hpart (in block order); if Hacc, also Hacc += H.
__global__ void k_proj_reduce(const double *__restrict__ Hpart, int nblk, int nv, int b, double *__restrict__ H,
                              int64_t ldh, double *__restrict__ Hacc, int64_t ldacc) {
    const int64_t total = (int64_t)nv * b;
    for (int64_t e = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; e < total;
         e += (int64_t)blockDim.x * gridDim.x) {
        double s0 = 0.0, s1 = 0.0;
        int q = 0;
        for (; q + 1 < nblk; q += 2) {
            s0 += Hpart[(int64_t)q * total + e];
            s1 += Hpart[(int64_t)(q + 1) * total + e];
        }
        if (q < nblk) s0 += Hpart[(int64_t)q * total + e];
        const double s = s0 + s1;
        const int r = (int)(e % nv), c = (int)(e / nv);
        H[r + (int64_t)c * ldh] = s;
        if (Hacc) Hacc[r + (int64_t)c * ldacc] += s;
    }
}

// W[rows] -= V[rows] H for the 64-row groups g = blockIdx.x, blockIdx.x +
// gridDim.x, ...: wave w takes rows 16 w .. 16 w + 15 of a group.
__global__ __launch_bounds__(256) void k_proj_update(const double *__restrict__ V, int64_t ldv, int nv,
                                                     const double *__restrict__ H, int64_t ldh,
                                                     double *__restrict__ W, int64_t ldw, int b, int64_t m) {
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int nJ = (b + 15) / 16;
    const int64_t groups = (m + 63) / 64;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t r0 = 64 * g + 16 * w;
        if (r0 >= m) continue;
        d4 acc[4];
#pragma unroll
        for (int J = 0; J < 4; ++J) acc[J] = d4_zero();
        const int64_t row = r0 + i;
        const bool rok = row < m;
#pragma unroll 4
        for (int k0 = 0; k0 < nv; k0 += 4) {
            // A[i][kq] = V[r0 + i][k0 + kq], B[kq][j] = H[k0 + kq][16 J + j]
            const int kk = k0 + kq;
            const bool kok = kk < nv;
            const double a = (rok && kok) ? V[row + (int64_t)kk * ldv] : 0.0;
#pragma unroll
            for (int J = 0; J < 4; ++J) {
                if (J < nJ) {
                    const int col = 16 * J + i;
                    const double h = (kok && col < b) ? H[kk + (int64_t)col * ldh] : 0.0;
                    acc[J] = mfma_f64(a, h, acc[J]);
                }
            }
        }
#pragma unroll
        for (int J = 0; J < 4; ++J) {
            if (J >= nJ) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t rw = r0 + d_row(q, lane);
                const int col = 16 * J + d_col(lane);
                if (rw < m && col < b) W[rw + (int64_t)col * ldw] -= acc[J][q];
            }
        }
    }
}

}  // namespace

int proj_blocks(int64_t m) {
    // rows per block a multiple of 16, about 4096 rows per block, at most
    // kProjMaxBlocks blocks
    int64_t nb = (m + 4095) / 4096;
    if (nb > kProjMaxBlocks) nb = kProjMaxBlocks;
    return (int)(nb < 1 ? 1 : nb);
}

hipError_t launch_proj(const double *V, int64_t ldv, int nv, const double *W, int64_t ldw, int b, int64_t m,
                       double *Hpart, double *H, int64_t ldh, double *Hacc, int64_t ldacc, hipStream_t st) {
    const int nblk = proj_blocks(m);
    const int64_t per = ((m + nblk - 1) / nblk + 15) / 16 * 16;
    {
        ProfScope ps("orth_proj_partial", st);
        hipLaunchKernelGGL(k_proj_partial, dim3((unsigned)nblk, (unsigned)((nv + kProjSlice - 1) / kProjSlice)),
                           dim3(256), 0, st, V, ldv, nv, W, ldw, b, m, per, Hpart);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ProfScope ps("orth_proj_reduce", st);
    const int64_t total = (int64_t)nv * b;
    const unsigned grid = (unsigned)((total + 255) / 256 < 1024 ? (total + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_proj_reduce, dim3(grid < 1 ? 1 : grid), dim3(256), 0, st, Hpart, nblk, nv, b, H, ldh,
                       Hacc, ldacc);
    return hipGetLastError();
}

hipError_t launch_proj_update(const double *V, int64_t ldv, int nv, const double *H, int64_t ldh, double *W,
                              int64_t ldw, int b, int64_t m, hipStream_t st) {
    ProfScope ps("orth_proj_update", st);
    const int64_t groups = (m + 63) / 64;
    const unsigned grid = (unsigned)(groups < 2048 ? groups : 2048);
    hipLaunchKernelGGL(k_proj_update, dim3(grid), dim3(256), 0, st, V, ldv, nv, H, ldh, W, ldw, b, m);
    return hipGetLastError();
}

}  // namespace tsqr
