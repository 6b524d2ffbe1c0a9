// factor_common.h -- device pieces shared by the leaf kernels (factor.hip)
// and the tree kernels (tree.hip): the workgroup shape, the LDS layout of a
// running triangle and its compact-WY factor, and the blocked T build.
#pragma once

#include "common.h"
#include "mfma.h"

namespace tsqr {

constexpr int kWaves = 4;                  // waves per tree workgroup (and narrow leaves)
constexpr int kFactorThreads = 64 * kWaves;
constexpr int kRowGroups = 4 * kWaves;     // row groups per 4-wave workgroup

// LDS of the leaf and tree kernels with W waves per workgroup (about 75 KiB
// for 4 waves, 83 KiB for 8).
template <int W>
struct FactorSmemT {
    double R[64 * kLdsStride];   // running triangle, row-major
    double T[64 * kLdsStride];   // upper: T of the chunk; strictly lower: Gram G^T
    union {
        struct {
            double red[2][64][W];    // per-wave partial dots, double-buffered
            double redq[2][64][W];   // per-wave pivot-row values (first chunk only)
        } s;
        double P[64 * 16];           // scratch of the blocked T build
    } u;
    double tau[64];
    double scl[64];   // reflector scale s_j of a later chunk's column j
};
using FactorSmem = FactorSmemT<kWaves>;

// Gram entry G[k][j] = y_k . y_j (k < j), kept in the lower triangle of T.
template <typename SM>
__device__ __forceinline__ double &gram(SM &sm, int k, int j) { return sm.T[j * kLdsStride + k]; }

// The LDS that build_t alone needs (T with the Gram entries below it, the
// block scratch, tau): about 42 KiB, so that T builds can share a CU with
// a tree combine's workgroup.
struct TBuildSmem {
    double T[64 * kLdsStride];
    union {
        double P[64 * 16];
    } u;
    double tau[64];
};

// Compact-WY factor T of the chunk (Sec. 2.2: H_1...H_n = I - V T V^T),
// built once per chunk from tau and the Gram matrix G = Y^T Y by the
// forward (Schreiber-Van Loan) recurrence T[0:j, j] = -tau_j T[0:j, 0:j]
// G[0:j, j], T_jj = tau_j, in 16-column blocks: wave J runs the recurrence
// inside diagonal block J in registers, then the off-diagonal blocks follow
// from the block form of the same recurrence,
//     T[0:16J, J] = -T[0:16J, 0:16J] (G[0:16J, J] T_JJ),
// as FP64 MFMA tiles.
// Waves past the fourth (8-wave leaves) take part in the barriers only.
template <typename SM>
__device__ __forceinline__ void build_t(SM &sm, const int n) {
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int j0 = 16 * w;
    double trow[16];
    const int i = lane & 15;
#pragma unroll
    for (int q = 0; q < 16; ++q) trow[q] = 0.0;
    if (j0 < n) {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = j0 + jj;
            if (j < n) {
                const double tj = sm.tau[j];
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < jj; ++q) acc = fma(trow[q], gram(sm, j0 + q, j), acc);
                trow[jj] = (i < jj) ? -tj * acc : ((i == jj) ? tj : 0.0);
            }
        }
    }
    __syncthreads();   // every wave has read its Gram block before T overwrites
    if (j0 < n && lane < 16) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (q >= i) sm.T[(j0 + i) * kLdsStride + j0 + q] = trow[q];
    }
    __syncthreads();
    for (int J = 1; J < 4 && 16 * J < n; ++J) {
        if (w < J) {   // P[16w : 16w + 16, :] = G[16w.., J block] T_JJ
            d4 acc = d4_zero();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const int kk = 4 * kb + (lane >> 4), jj = lane & 15;
                const int k = 16 * J + kk;
                const double t = (kk <= jj) ? sm.T[k * kLdsStride + 16 * J + jj] : 0.0;
                acc = mfma_f64(gram(sm, 16 * w + (lane & 15), k), t, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.u.P[(16 * w + d_row(r, lane)) * 16 + d_col(lane)] = acc[r];
        }
        __syncthreads();
        if (w < J) {   // T[16w.., J block] = -T[16w.., 0:16J] P
            d4 acc = d4_zero();
            const int row = 16 * w + (lane & 15);
            for (int kb = 4 * w; kb < 4 * J; ++kb) {
                const int k = 4 * kb + (lane >> 4);
                const double t = (k >= row) ? sm.T[row * kLdsStride + k] : 0.0;
                acc = mfma_f64(t, sm.u.P[k * 16 + (lane & 15)], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sm.T[(16 * w + d_row(r, lane)) * kLdsStride + 16 * J + d_col(lane)] = -acc[r];
        }
        __syncthreads();
    }
}

typedef double dv2 __attribute__((ext_vector_type(2)));


// Value of v in lane `src` (uniform across the wave).
__device__ __forceinline__ double read_lane(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Upper triangle of an LDS matrix (row-major) -> column-major n x n with
// zeros below the diagonal.
__device__ __forceinline__ void store_tri(const double *lds, double *__restrict__ dst, int n) {
    for (int e = local_tid(); e < n * n; e += (int)blockDim.x) {
        const int r = e % n, k = e / n;
        dst[e] = (r <= k) ? lds[r * kLdsStride + k] : 0.0;
    }
}

__device__ __forceinline__ void zero_lds(double *lds) {
    for (int e = threadIdx.x; e < 64 * kLdsStride; e += blockDim.x) lds[e] = 0.0;
}

// Gram entries and tau of a chunk's or a tree node's reflectors, for its T
// (built later by node_t):
// dst (n x n, column-major) gets G[c][r] = y_c . y_r at (r, c) for r > c
// and tau_r at (r, r).
__device__ __forceinline__ void store_gram(const FactorSmem &sm, double *__restrict__ dst, int n) {
    for (int e = threadIdx.x; e < n * n; e += kFactorThreads) {
        const int r = e % n, c = e / n;
        dst[e] = (r > c) ? sm.T[r * kLdsStride + c] : ((r == c) ? sm.tau[r] : 0.0);
    }
}

// T from the Gram entries and tau that store_gram left in Tn, by the
// forward recurrence of build_t; T overwrites them.
__device__ __forceinline__ void node_t(FactorSmem &sm, double *__restrict__ Tn, int n) {
    // build_t's block products read Gram entries of the last 16-column block
    // past n (times zero) when n is not a multiple of 16
    if (n % 16 != 0) {
        zero_lds(sm.T);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n * n; e += kFactorThreads) {
        const int r = e % n, c = e / n;
        const double v = Tn[e];
        if (r > c) sm.T[r * kLdsStride + c] = v;
        else if (r == c) sm.tau[r] = v;
    }
    __syncthreads();
    build_t(sm, n);
    store_tri(sm.T, Tn, n);
}

}  // namespace tsqr
