// mfma.h -- FP64 matrix-core tiles for gfx950 (v_mfma_f64_16x16x4f64).
//
// One instruction computes D(16x16) += A(16x4) B(4x16) on a wave:
//   A[i][k] is held by lane i + 16 k,
//   B[k][j] is held by lane j + 16 k,
//   D[i][j] is register (i / 4) of lane j + 16 (i % 4).
// (Layout measured on the device with a one-wave probe.)
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace tsqr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4_zero() {
    d4 z = {0.0, 0.0, 0.0, 0.0};
    return z;
}

// FP32 tile (v_mfma_f32_16x16x4f32): A and B as above; D[i][j] is register
// (i % 4) of lane j + 16 (i / 4) -- a different output layout from FP64.
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Precision traits of the 16x16x4 tiles: element type, accumulator vector
// and the row of D held in register r of lane l.
struct TileF64 {
    using T = double;
    using Acc = d4;
    __device__ static Acc mfma(T a, T b, Acc c) { return mfma_f64(a, b, c); }
    __device__ static int drow(int r, int lane) { return 4 * r + (lane >> 4); }
};
struct TileF32 {
    using T = float;
    using Acc = f4;
    __device__ static Acc mfma(T a, T b, Acc c) { return mfma_f32(a, b, c); }
    __device__ static int drow(int r, int lane) { return 4 * (lane >> 4) + r; }
};

// Row of a FP64 D held in register r of lane l, and its column.
__device__ __forceinline__ int d_row(int r, int lane) { return 4 * r + (lane >> 4); }
__device__ __forceinline__ int d_col(int lane) { return lane & 15; }

// C = op(A) * B for 64 x 64 row-major LDS matrices (row stride ld),
// computed by the 4 waves of a 256-thread workgroup: wave w produces the
// 16-row block w of C.  `a_upper` skips the zero blocks of an upper-
// triangular A.  If transA, op(A) = A^T.  C may not alias A or B.
__device__ __forceinline__ void lds_gemm64(const double *A, const double *B, double *C, int ld,
                                           bool a_upper, bool transA, double scale) {
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int I = w;
    d4 acc[4];
#pragma unroll
    for (int J = 0; J < 4; ++J) acc[J] = d4_zero();
    // op(A) upper triangular: blocks K < I vanish
    const int kb0 = a_upper ? 4 * I : 0;
    for (int kb = kb0; kb < 16; ++kb) {
        const int i = 16 * I + (lane & 15), k = 4 * kb + (lane >> 4);
        const double a = transA ? A[k * ld + i] : A[i * ld + k];
#pragma unroll
        for (int J = 0; J < 4; ++J) acc[J] = mfma_f64(a, B[k * ld + 16 * J + (lane & 15)], acc[J]);
    }
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            C[(16 * I + d_row(r, lane)) * ld + 16 * J + d_col(lane)] = scale * acc[J][r];
}

}  // namespace tsqr
