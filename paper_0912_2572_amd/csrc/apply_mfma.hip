// apply_mfma.hip -- leaf part of Q^T B / Q B on FP64 matrix cores, for
// blocks of up to 16 columns of B (least squares, refinement corrections).
//
// Per chunk of a domain (compact-WY factor I - Y T Y^T, Sec. 2.2):
//     W = Yb + V^T B_c          (Yb = the domain's top n rows; 0 on a first
//                                chunk, whose V has an implicit unit diagonal)
//     Z = T^T W  (Q^T)  or  T W  (Q)
//     Yb -= Z,   B_c -= V Z
// W is reduced over the chunk's rows by v_mfma_f64_16x16x4f64 with the row
// index as the reduction dimension (each wave takes a quarter of the rows,
// the four partials meet in LDS); the update runs transposed,
// (B_c - V Z)^T = B_c^T - Z^T V^T, so that each store writes 16 consecutive
// rows of a column.
#include "common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

constexpr int KBM = 16;   // columns of B per workgroup

struct ApplyMSmem {
    double T[64 * kLdsStride];
    double Wp[4][64][KBM];   // per-wave partials of W
    double W[64][KBM];
    double Y[64][KBM];       // the domain's top n rows of B (columns of this block)
};

// V element of a chunk with the implicit unit diagonal of a first chunk.
__device__ __forceinline__ double v_elem(const double *__restrict__ Vc, int64_t ldv, int64_t row, int col,
                                         int64_t valid, int n, bool first) {
    if (row >= valid || col >= n) return 0.0;
    if (first && row <= col) return (row == col) ? 1.0 : 0.0;
    return Vc[row + (int64_t)col * ldv];
}

__device__ void chunk_apply_m(ApplyMSmem &sm, const double *__restrict__ Vc, int64_t ldv,
                              const double *__restrict__ Tk, const double *__restrict__ Bin, int64_t ldbi,
                              double *__restrict__ Bout, int64_t ldbo, int64_t valid, int n, int kc,
                              bool first, int trans) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int mtn = (n + 15) >> 4;             // 16-reflector tiles
    // stage T (row-major)
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, q = e >> 6;
        sm.T[r * kLdsStride + q] = (r < n && q < n) ? Tk[r + (int64_t)q * n] : 0.0;
    }
    // W partial over this wave's rows: W[m][j] += sum_r V[r][m] B[r][j]
    {
        d4 acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = d4_zero();
        const int64_t per = ((valid + 15) / 16 + 3) / 4 * 16;   // rows per wave, multiple of 16
        const int64_t lo = w * per, hi = (lo + per < valid) ? lo + per : valid;
        for (int64_t r4 = lo; r4 < hi; r4 += 4) {
            const int64_t row = r4 + l4;
            double b = 0.0;
            if (row < hi && l16 < kc) {
                if (first && !trans && row < n) b = sm.Y[row][l16];
                else b = Bin[row + (int64_t)l16 * ldbi];
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                if (mt >= mtn) break;
                const double a = (row < hi) ? v_elem(Vc, ldv, row, 16 * mt + l16, valid, n, first) : 0.0;
                acc[mt] = mfma_f64(a, b, acc[mt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Wp[w][16 * mt + d_row(r, lane)][d_col(lane)] = acc[mt][r];
    }
    __syncthreads();
    for (int e = tid; e < 64 * KBM; e += 256) {
        const int m = e >> 4, j = e & 15;
        double s = ((sm.Wp[0][m][j] + sm.Wp[1][m][j]) + sm.Wp[2][m][j]) + sm.Wp[3][m][j];
        if (!first) s += sm.Y[m][j];
        sm.W[m][j] = s;
    }
    __syncthreads();
    // Z = op(T) W, written over the partial buffer of wave 0
    for (int e = tid; e < 64 * KBM; e += 256) {
        const int i = e >> 4, j = e & 15;
        double z = 0.0;
        if (i < n) {
            if (trans) {
                for (int q = 0; q <= i; ++q) z = fma(sm.T[q * kLdsStride + i], sm.W[q][j], z);
            } else {
                for (int q = i; q < n; ++q) z = fma(sm.T[i * kLdsStride + q], sm.W[q][j], z);
            }
        }
        sm.Wp[0][i][j] = z;
    }
    __syncthreads();
    if (!first)
        for (int e = tid; e < 64 * KBM; e += 256) {
            const int i = e >> 4, j = e & 15;
            sm.Y[i][j] -= sm.Wp[0][i][j];
        }
    // B_c^T -= Z^T V^T over 16-row tiles: wave w takes tiles w, w + 4, ...
    const int kbn = (n + 3) >> 2;
    for (int64_t t0 = 16 * w; t0 < valid; t0 += 64) {
        const int64_t row = t0 + l16;
        d4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = 4 * r + l4;
            double b = 0.0;
            if (row < valid && col < kc) {
                if (first && !trans && row < n) b = sm.Y[row][col];
                else b = Bin[row + (int64_t)col * ldbi];
            }
            acc[r] = b;
        }
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
            if (kb >= kbn) break;
            const int k = 4 * kb + l4;
            const double a = -sm.Wp[0][k][l16];               // -Z^T[col l16][refl k]
            const double v = v_elem(Vc, ldv, row, k, valid, n, first);
            acc = mfma_f64(a, v, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = 4 * r + l4;
            if (row < valid && col < kc) {
                if (first && trans && row < n) sm.Y[row][col] = acc[r];
                else Bout[row + (int64_t)col * ldbo] = acc[r];
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_leaf_apply_m(const double *__restrict__ V, int64_t ldv,
                                                      const double *__restrict__ Tc, PanelArgs pa,
                                                      const double *__restrict__ Bsrc, int64_t ldbs,
                                                      double *__restrict__ B, int64_t ldb, int64_t k,
                                                      int trans) {
    extern __shared__ double smem_raw[];
    ApplyMSmem &sm = *reinterpret_cast<ApplyMSmem *>(smem_raw);
    const int64_t dom = blockIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * KBM;
    const int kc = (int)((k - c0 < KBM) ? k - c0 : KBM);
    const int n = pa.n;
    const int64_t row0 = dom * pa.mb;
    const int64_t nrows = (dom == pa.P - 1) ? pa.m - row0 : pa.mb;
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    const int64_t nn = (int64_t)n * n;
    const double *Bs0 = Bsrc + c0 * ldbs;
    double *B0 = B + c0 * ldb;
    const int tid = threadIdx.x;
    if (trans) {
        for (int64_t ch = 0; ch < nch; ++ch) {
            const int64_t r0 = row0 + ch * pa.chunk;
            const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
            chunk_apply_m(sm, V + r0, ldv, Tc + (dom * pa.cpd + ch) * nn, Bs0 + r0, ldbs, B0 + r0, ldb,
                          valid, n, kc, ch == 0, 1);
        }
        for (int e = tid; e < 64 * KBM; e += 256) {
            const int r = e >> 4, c = e & 15;
            if (r < n && c < kc) B0[row0 + r + (int64_t)c * ldb] = sm.Y[r][c];
        }
    } else {
        for (int e = tid; e < 64 * KBM; e += 256) {
            const int r = e >> 4, c = e & 15;
            sm.Y[r][c] = (r < n && c < kc) ? Bs0[row0 + r + (int64_t)c * ldbs] : 0.0;
        }
        __syncthreads();
        for (int64_t ch = nch - 1; ch >= 0; --ch) {
            const int64_t r0 = row0 + ch * pa.chunk;
            const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
            chunk_apply_m(sm, V + r0, ldv, Tc + (dom * pa.cpd + ch) * nn, Bs0 + r0, ldbs, B0 + r0, ldb,
                          valid, n, kc, ch == 0, 0);
        }
    }
}

hipError_t launch_leaf_apply_m(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                               const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                               int trans, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const size_t sh = sizeof(ApplyMSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_leaf_apply_m,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)pa.P, (unsigned)((k + KBM - 1) / KBM));
    ProfScope ps(trans ? "leaf_apply_qt" : "leaf_apply_q", st);
    hipLaunchKernelGGL(k_leaf_apply_m, grid, dim3(256), sh, st, V, ldv, Tc, pa, Bsrc, ldbs, B, ldb, k,
                       trans);
    return hipGetLastError();
}

}  // namespace tsqr
