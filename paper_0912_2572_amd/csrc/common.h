// common.h -- device helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tsqr {

// Row stride (in doubles) of the n x n triangles staged in LDS; odd so that
// reads down a column of the row-major copy hit distinct banks.
constexpr int kLdsStride = 65;

// Rows per thread of the leaf kernel's register tile for `ns` column slots
// per thread (8 * ns columns): 64 / ns, capped at 32 so the tile plus its
// broadcast copy of one column stays in registers.
__host__ __device__ constexpr int rows_per_thread(int ns) { return ns >= 2 ? 64 / ns : 32; }

// Sum over the 8 lanes that share a column group (lane = rg * 8 + cg), i.e.
// across lane bits 3..5.  Butterfly with commutative pairwise adds, so every
// participating lane ends with the bitwise-identical sum.
__device__ __forceinline__ double sum_rowgroups(double v) {
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// Householder scalars for x = [alpha; x2] with ||x2||^2 = sig2 (Sec. 2.2,
// H = I - tau v v^T, LAPACK's sign convention, sgn(0) = +1):
//   beta = -sgn(alpha) sqrt(alpha^2 + sig2), tau = (beta - alpha) / beta,
//   v = [1; x2 * s] with s = 1 / (alpha - beta).
// sig2 == 0 gives H = I (tau = 0, beta = alpha, s = 0).
__device__ __forceinline__ void householder_scalars(double alpha, double sig2, double &beta,
                                                    double &tau, double &s) {
    if (sig2 == 0.0) {
        beta = alpha;
        tau = 0.0;
        s = 0.0;
        return;
    }
    const double sgn = (alpha < 0.0) ? -1.0 : 1.0;
    beta = -sgn * sqrt(alpha * alpha + sig2);
    tau = (beta - alpha) / beta;
    s = 1.0 / (alpha - beta);
}

}  // namespace tsqr
