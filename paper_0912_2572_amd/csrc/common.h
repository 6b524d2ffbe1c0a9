// common.h -- device helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tsqr {

// Row stride (in doubles) of the n x n triangles staged in LDS; odd so that
// reads down a column of the row-major copy hit distinct banks.
constexpr int kLdsStride = 65;

// Leaf register tile: 16 column groups x 4 row groups per wave (lane =
// 16 rg + cg), `ns` column slots per thread (16 ns columns) and
// rows_per_thread(ns) rows per thread; 16 row groups per 256-thread
// workgroup, so a chunk has 16 * rows_per_thread(ns) rows.
__host__ __device__ constexpr int rows_per_thread(int ns) { return ns >= 2 ? 16 : 32; }
__host__ __device__ constexpr int chunk_rows(int ns) { return 16 * rows_per_thread(ns); }

// The thread index, hidden from the optimizer: values derived from it are
// then computed where they are used instead of being hoisted out of outer
// loops, which under full register files only spills them.
__device__ __forceinline__ int local_tid() {
    int v = (int)threadIdx.x;
    asm volatile("" : "+v"(v));
    return v;
}

// 64-bit lane permutations built from 32-bit DPP / swizzle primitives.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int PATTERN>
__device__ __forceinline__ double swizzle_f64(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), PATTERN);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), PATTERN);
    return __hiloint2double(hi, lo);
}
constexpr int kDppRowRor8 = 0x128;     // lane i <- lane (i + 8) mod 16 of its row = i ^ 8
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kSwizzleXor16 = 0x401F;  // bit mode: and 0x1f, xor 0x10

// v[l & ~16] + v[l | 16] for every lane (exchange across lane bit 4), the
// same sum in the same order on both lanes of a pair.
__device__ __forceinline__ double pair_sum16(double v) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// v[l & ~32] + v[l | 32] (exchange across lane bit 5).
__device__ __forceinline__ double pair_sum32(double v) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Two pair sums for the price of one exchange: a lane with bit 4 clear ends
// with a[l] + a[l ^ 16], a lane with bit 4 set with b[l] + b[l ^ 16] (the
// swap trades the odd 16-lane rows of its first operand for the even rows of
// its second).  Each total is bitwise the one pair_sum16 gives.
__device__ __forceinline__ double split_sum16(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// Across lane bit 5: lanes 0..31 end with a[l] + a[l ^ 32], lanes 32..63
// with b[l] + b[l ^ 32].
__device__ __forceinline__ double split_sum32(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Wave total of per-slot partials p[t] (t < NS, NS in {1, 2, 4}) over the 4
// 16-lane rows, returned in row r for slot r (r < NS): one exchange tree for
// all slots instead of one per slot.
template <int NS>
__device__ __forceinline__ double row_slot_total(const double (&p)[NS]) {
    static_assert(NS == 1 || NS == 2 || NS == 4, "slot count");
    if constexpr (NS == 4) return split_sum32(split_sum16(p[0], p[1]), split_sum16(p[2], p[3]));
    else if constexpr (NS == 2) return pair_sum32(split_sum16(p[0], p[1]));
    else return pair_sum32(pair_sum16(p[0]));
}

// Sum over the 8 lanes that share a column group (lane = rg * 8 + cg), i.e.
// across lane bits 3..5, entirely in the VALU (DPP and permlane swaps).
// Every participating lane ends with the bitwise-identical sum.
__device__ __forceinline__ double sum_rowgroups(double v) {
    v += dpp_f64<kDppRowRor8>(v);
    v = pair_sum16(v);
    v = pair_sum32(v);
    return v;
}

// Sum over the 4 lanes of a quad (lane bits 0..1), identical in all four.
__device__ __forceinline__ double sum_quad(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
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
    // r = 1 / sqrt(alpha^2 + sig2) from v_rsq_f64 and two Newton steps
    // r <- r (3 - x r^2) / 2, so that |beta| = x r and 1 / beta = -sgn r come
    // from one short chain (no square root expansion, no reciprocal of beta)
    const double x = fma(alpha, alpha, sig2);
    // (x is a normal number over the library's supported magnitudes,
    // 2^-400 .. 2^400, so r^2 stays finite)
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    r = r * fma(-hx, r * r, 1.5);
    r = r * fma(-hx, r * r, 1.5);
    beta = -sgn * (x * r);
    // s = 1 / (alpha - beta): v_rcp_f64 and two Newton steps r <- r + r (1 - d r);
    // tau = (beta - alpha) / beta = -(alpha - beta) / beta = sgn (alpha - beta) r
    const double d = alpha - beta;
    double rd = __builtin_amdgcn_rcp(d);
    rd = fma(rd, fma(-d, rd, 1.0), rd);
    rd = fma(rd, fma(-d, rd, 1.0), rd);
    s = rd;
    tau = sgn * (d * r);
}

// ---- one-wave triangular solves for n <= 256 (column-major R, ld n) ----
// Lane l holds entries l + 64 q in xr[q], q < 4.  No barrier: the wave
// broadcasts each solved entry with a lane read.  The columns (or rows) of R
// and their diagonal entries are fetched kSolveAhead steps ahead into a ring
// of registers, so a step waits on a load issued several steps earlier
// instead of a full memory latency.  Every load address is clamped into R
// (out-of-range entries are loaded from R[0..] and replaced by zero), so the
// loads are unconditional.

constexpr int kSolveAhead = 4;

__device__ __forceinline__ double wave_bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double pick4(const double (&xr)[4], int q) {
    return q == 0 ? xr[0] : (q == 1 ? xr[1] : (q == 2 ? xr[2] : xr[3]));
}

// Back substitution R x = b (b in xr on entry, x on exit).
__device__ __forceinline__ void wave_backsub(const double *__restrict__ R, int n, double (&xr)[4]) {
    if (n <= 0) return;
    const int lane = threadIdx.x & 63;
    constexpr int D = kSolveAhead;
    double col[D][4], dg[D];
    // column j above the diagonal and R[j][j]; j < 0 loads column 0 (unused)
    auto fetch = [&](int j, double (&cc)[4], double &d) {
        const int jj = j < 0 ? 0 : j;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = lane + 64 * q;
            const double v = R[(i < jj ? i : 0) + (int64_t)jj * n];
            cc[q] = (i < jj) ? v : 0.0;
        }
        d = R[jj + (int64_t)jj * n];
    };
    auto step = [&](int j, const double (&cc)[4], double d) {
        const int qj = j >> 6, lj = j & 63;
        const double xj = wave_bcast(pick4(xr, qj), lj) / d;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
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

// Forward substitution R^T h = g (g in xr on entry, h on exit).
__device__ __forceinline__ void wave_fwdsub_t(const double *__restrict__ R, int n, double (&xr)[4]) {
    if (n <= 0) return;
    const int lane = threadIdx.x & 63;
    constexpr int D = kSolveAhead;
    double row[D][4], dg[D];
    // row i right of the diagonal (R[i][c], i < c < n) and R[i][i];
    // i >= n loads row 0 (unused)
    auto fetch = [&](int i, double (&rr)[4], double &d) {
        const int ii = i < n ? i : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = lane + 64 * q;
            const bool in = c > ii && c < n;
            const double v = R[ii + (int64_t)(in ? c : ii) * n];
            rr[q] = in ? v : 0.0;
        }
        d = R[ii + (int64_t)ii * n];
    };
    auto step = [&](int i, const double (&rr)[4], double d) {
        const int qi = i >> 6, li = i & 63;
        const double hi = wave_bcast(pick4(xr, qi), li) / d;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xr[q] = fma(-rr[q], hi, xr[q]);
            if (q == qi && lane == li) xr[q] = hi;
        }
    };
#pragma unroll
    for (int u = 0; u < D; ++u) fetch(u, row[u], dg[u]);
    int i0 = 0;
    for (; i0 + (D - 1) < n; i0 += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            step(i0 + u, row[u], dg[u]);
            fetch(i0 + u + D, row[u], dg[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < D - 1; ++u)
        if (i0 + u < n) step(i0 + u, row[u], dg[u]);
}

// Sum over the 64 lanes, identical in every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v = sum_quad(v);                      // lanes within 4
    v += __shfl_xor(v, 4);                // the two quads of 8 lanes
    v += dpp_f64<kDppRowRor8>(v);         // the two halves of a 16-lane row
    v = pair_sum16(v);
    v = pair_sum32(v);
    return v;
}

}  // namespace tsqr
