// factor.hip -- leaf kernels of the TSQR factorization on gfx950 (the tree
// kernels are in tree.hip).
//
// Leaf (Sec. 2.3, "the factorization of a domain is the operation performed
// on the leaves"): one 256-thread workgroup per domain.  The domain is
// streamed from HBM in chunks that live in registers; the domain's triangle
// R lives in LDS.  The first chunk gets a plain Householder QR (its top n
// rows become R); every later chunk C gets the structured QR of [R; C] --
// the paper's flat tree (Sec. 2.3) applied inside the domain, so A is read
// exactly once.  Each chunk leaves its reflectors V in place of the chunk
// and its compact-WY factor T (Sec. 2.2: H_1...H_n = I - V T V^T).
//
// Register tile of a chunk: 256 threads (4 waves); lane = 16 rg + cg (cg =
// column group 0..15, rg = row group 0..3 inside the wave, 16 row groups per
// workgroup).  A thread owns rows {RPT (4 w + rg) + i : i < RPT} and columns
// {cg + 16 t : t < NS}.  Column step j of Householder QR needs one reduction: with x = column
// j, the dots d_k = x . c_k for every column k give ||x||^2 (k = j), the
// update coefficients (k > j) and, for k < j, the Gram entries y_k . y_j
// that build T.  The reduction over the 4 row groups of a wave runs in the
// VALU (lane permutes); the 4 waves meet at one barrier per step.
#include <type_traits>
#include <utility>

#include "common.h"
#include "factor_common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

// Thread index as the step code uses it: for narrow panels (NS <= 2, two
// workgroups per CU, 256 registers) hidden from the optimizer so that
// loop-invariant addresses are not hoisted into spills; the wide kernel has
// the AGPRs to keep them.
template <int NS>
__device__ __forceinline__ int step_tid() { return NS == 2 ? local_tid() : (int)threadIdx.x; }

// G[k][j] (k < j) at step j from d = x . c_k, with s = s_j.  First chunk:
// c_k is the scaled reflector y_k below the pivot rows and e its pivot-row
// entry, so G = e + s d.  Later chunk: the reflector column c_k is still
// unscaled (y_k = [e_k; s_k c_k]) and y_k, y_j share no R-part entry, so
// G = s_k (s d).
template <bool FIRST, int W>
__device__ __forceinline__ double gram_entry(const FactorSmemT<W> &sm, int k, double s, double d, double e) {
    if constexpr (FIRST) return fma(s, d, e);
    else return sm.scl[k] * (s * d);
}

// Half of a full chunk's reflectors (slots 2 and 3: columns 32..63) of the
// wide FP64 kernel, parked in LDS at the end of the chunk and copied out in
// four parts at the starts of the next chunk's four column slots: the V
// stores then drain while the column steps run (they issue no other memory
// traffic) instead of all 256 CUs storing 32 MB at once at the chunk's end.
// Passed by value (dst == nullptr: nothing staged), so that its uniform
// fields stay in scalar registers.
constexpr int kStageLd = 256 + 2;   // doubles per staged column (padded against bank conflicts)
constexpr size_t kStageBytes = sizeof(double) * 32 * kStageLd;

struct Drain {
    const double *stage;   // LDS, column cl (0..31) at stage + cl * kStageLd
    double *dst;           // row 0 of the staged chunk's V, or nullptr
    int64_t ld;
    int n;
};

// Slots 2 and 3 of a 256-row chunk (RPT = 16) into the stage.
__device__ __forceinline__ void stage_slots(double *stage, const double (&c)[16][4]) {
    const int tid = local_tid(), w = tid >> 6, lane = tid & 63, cg = lane & 15, rg = lane >> 4;
    const int rgw = w * 4 + rg;
#pragma unroll
    for (int t = 2; t < 4; ++t) {
        double *base = stage + (cg + 16 * (t - 2)) * kStageLd + 16 * rgw;
#pragma unroll
        for (int i = 0; i < 16; i += 2) {
            dv2 v;
            v.x = c[i][t];
            v.y = c[i + 1][t];
            *reinterpret_cast<dv2 *>(base + i) = v;
        }
    }
}

// Part p (0..3) of the staged columns: 32 + 8p .. 32 + 8p + 7; per store a
// thread moves rows 2 (tid % 128), +1 of one column (16 bytes).
__device__ __forceinline__ void drain_part(const Drain d, int p) {
    const int tid = local_tid(), half = tid >> 7, rp = 2 * (tid & 127);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int cl = 8 * p + 2 * i + half;
        if (32 + cl < d.n) {
            const dv2 v = *reinterpret_cast<const dv2 *>(d.stage + cl * kStageLd + rp);
            *reinterpret_cast<dv2 *>(d.dst + rp + (int64_t)(32 + cl) * d.ld) = v;
        }
    }
}

// State carried across the column steps of one chunk.
template <int NS, int RPT>
struct StepState {
    double rnew[NS];     // new R row, written one step late
    double xa[RPT];      // current / next column (ping-pong)
    double xb[RPT];
    int jprev = -1;
};

// Total of column k over the waves' partials, in a fixed order, so every
// thread that needs column k's total computes the same bits.
template <int W>
__device__ __forceinline__ double col_total(const double (&a)[2][64][W], int par, int k) {
    const double2 *p = reinterpret_cast<const double2 *>(&a[par][k][0]);
    double2 v[W / 2];
#pragma unroll
    for (int h = 0; h < W / 2; ++h) v[h] = p[h];
    double s = v[0].x + v[0].y;
#pragma unroll
    for (int h = 1; h < W / 2; ++h) s = (s + v[h].x) + v[h].y;
    return s;
}

// Column step j (= 16 TJ + q) of chunk_qr.  TJ is a template parameter so
// that the slot index of column j is known at compile time.
//
// With x = column j (rows of a first chunk above the pivot are 0, the pivot
// row itself is left out), one reduction gives d_k = x . c_k for every
// column k; then with alpha (the R entry or the pivot value) the Householder
// scalars follow and
//     k > j:  w = e_k + s d_k,  c_k -= tau w s x,  R[j][k] = e_k - tau w
//     k = j:  v_j = s x,  R[j][j] = beta
//     k < j:  G[k][j] = y_k . y_j = (pivot-row value) + s d_k.
// In a later chunk the reflector column keeps x and s is applied once at
// the end of the chunk, so there G[k][j] = s_k s d_k.
// The next column's pre-update values are fetched into xn from their owner
// lanes before the barrier, and every thread applies step j's update to
// them itself (the same fma as the owner), so the next step needs no
// shuffle on its critical path.
template <int NS, int RPT, int TJ, bool FIRST, int W>
__device__ __forceinline__ void one_step(const int j, const int q, double (&c)[RPT][NS],
                                         const int n, FactorSmemT<W> &sm, const bool want_t,
                                         double (&x)[RPT], double (&xn)[RPT], double (&rnew)[NS],
                                         int &jprev) {
    const int tid = step_tid<NS>();
    const int w = tid >> 6, lane = tid & 63, cg = lane & 15, rg = lane >> 4;
    const int rgw = w * 4 + rg;
    const int par = j & 1;
    // first chunk: row j is the pivot row, reduced separately (qv) and left
    // out of the dots.  Lane-dependent choices below are selects, not
    // branches, so the wave keeps one execution mask.
    const bool own_j = FIRST && (rgw == j / RPT);
    const int ij = j % RPT;
    double qv[NS];
    if (FIRST) {
#pragma unroll
        for (int t = 0; t < NS; ++t) qv[t] = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const bool piv = own_j && (i == ij);
#pragma unroll
            for (int t = 0; t < NS; ++t) qv[t] = piv ? c[i][t] : qv[t];
            x[i] = piv ? 0.0 : x[i];
        }
    }
    // prefetch column j + 1 (pre-update) from its owner lane
    if (q < 15) {
        const int src = (rg << 4) | (q + 1);
#pragma unroll
        for (int i = 0; i < RPT; ++i) xn[i] = __shfl(c[i][TJ], src);
    } else if constexpr (TJ + 1 < NS) {
        const int src = rg << 4;
#pragma unroll
        for (int i = 0; i < RPT; ++i) xn[i] = __shfl(c[i][TJ + 1], src);
    } else {
#pragma unroll
        for (int i = 0; i < RPT; ++i) xn[i] = 0.0;
    }
    // dots, the NS slots' accumulator chains interleaved; lane (cg, rg)
    // publishes the wave's partial of column cg + 16 rg
    {
        double s0[NS], s1[NS], p[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            s0[t] = 0.0;
            s1[t] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < RPT; i += 2) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                s0[t] = fma(x[i], c[i][t], s0[t]);
                s1[t] = fma(x[i + 1], c[i + 1][t], s1[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) p[t] = s0[t] + s1[t];
        const double pub = row_slot_total<NS>(p);
        double pubq = 0.0;
        if constexpr (FIRST) pubq = row_slot_total<NS>(qv);
        if (rg < NS) {
            sm.u.s.red[par][cg + 16 * rg][w] = pub;
            if (FIRST) sm.u.s.redq[par][cg + 16 * rg][w] = pubq;
        }
    }
    // non-first chunk: row j of the running R is final until this step's
    // deferred write (after the next barrier), so it is read before the
    // barrier, off the critical path
    double alpha = 0.0, en = 0.0, ev[NS];
    if (!FIRST) {
        alpha = sm.R[j * kLdsStride + j];
        en = (j + 1 < n) ? sm.R[j * kLdsStride + j + 1] : 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) ev[t] = sm.R[j * kLdsStride + cg + 16 * t];
    }
    __syncthreads();
    // deferred write of the previous step's R row: every thread has read
    // that row before this barrier.
    if (jprev >= 0 && rgw == 0) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 16 * t;
            if (k >= jprev) sm.R[jprev * kLdsStride + k] = rnew[t];
        }
    }
    // this thread's columns: dots d and (first chunk) the pivot-row entries
    // e.  Narrow kernels: each thread sums its own columns straight from LDS
    // (one LDS round trip on the critical path), and column j's values sit
    // in slot TJ of lane q, column j + 1's in lane q + 1 or, past the slot,
    // lane 0 of slot TJ + 1.  Wide kernel (no registers for that): lane k
    // sums column k and the threads fetch their columns from those lanes.
    double dv[NS];
    const bool has_next = j + 1 < n;
    double tot = 0.0, totq = 0.0;
    if constexpr (NS <= 2) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            dv[t] = col_total(sm.u.s.red, par, cg + 16 * t);
            if (FIRST) ev[t] = col_total(sm.u.s.redq, par, cg + 16 * t);
        }
    } else {
        tot = col_total(sm.u.s.red, par, threadIdx.x & 63);
        totq = FIRST ? col_total(sm.u.s.redq, par, threadIdx.x & 63) : 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            dv[t] = __shfl(tot, cg + 16 * t);
            if (FIRST) ev[t] = __shfl(totq, cg + 16 * t);
        }
    }
    // column j's and j + 1's values: lanes j and j + 1 of tot (wide), or
    // slot TJ of lanes q and q + 1, past the slot lane 0 of slot TJ + 1
    auto at_j = [&](const double (&v)[NS], double whole) -> double {
        if constexpr (NS <= 2) return read_lane(v[TJ], q);
        else return read_lane(whole, j);
    };
    auto at_next = [&](const double (&v)[NS], double whole) -> double {
        if constexpr (NS > 2) return read_lane(whole, j + 1);
        else if constexpr (TJ + 1 < NS) return q < 15 ? read_lane(v[TJ], q + 1) : read_lane(v[TJ + 1], 0);
        else return read_lane(v[TJ], q < 15 ? q + 1 : q);
    };
    const double sig2 = at_j(dv, tot);
    const double dn = has_next ? at_next(dv, tot) : 0.0;
    if (FIRST) {
        alpha = at_j(ev, totq);
        if (has_next) en = at_next(ev, totq);
    }
    double beta, tau, s;
    householder_scalars(alpha, sig2, beta, tau, s);
    // the next column after this step's update (same fma as its owner)
    {
        const double fn = (tau * fma(s, dn, en)) * s;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const double u = fma(-fn, x[i], xn[i]);
            xn[i] = (FIRST && own_j && i == ij) ? 0.0 : u;
        }
    }
    // trailing update (k > j), reflector (k == j), Gram entries (k < j).
    // Slots t < TJ hold only columns k < j and slots t > TJ only k > j
    // (both known at compile time); slot TJ mixes all three by lane.
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int k = cg + 16 * t;
        const double d = dv[t];
        const double e = ev[t];
        if (t < TJ) {
            if (want_t && rgw == 0) gram(sm, k, j) = gram_entry<FIRST, W>(sm, k, s, d, e);
            continue;
        }
        const double wv = fma(s, d, e);
        if (t > TJ) {
            const double f = (tau * wv) * s;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const double u = fma(-f, x[i], c[i][t]);
                c[i][t] = (FIRST && own_j && i == ij) ? 0.0 : u;
            }
            rnew[t] = e - tau * wv;
        } else {
            const bool upd = cg > q, refl = cg == q;
            const double f = upd ? (tau * wv) * s : 0.0;
            if constexpr (FIRST) {
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double u = fma(-f, x[i], c[i][t]);
                    const double r = refl ? s * x[i] : u;
                    c[i][t] = (own_j && upd && i == ij) ? 0.0 : r;
                }
            } else {
                // the reflector column keeps x (bitwise its owner's column);
                // its scale s waits in sm.scl for the end of the chunk
#pragma unroll
                for (int i = 0; i < RPT; ++i) c[i][t] = fma(-f, x[i], c[i][t]);
            }
            rnew[t] = upd ? e - tau * wv : beta;
            if (want_t && rgw == 0 && cg < q) gram(sm, k, j) = gram_entry<FIRST, W>(sm, k, s, d, e);
        }
    }
    if (tid == 0) {
        sm.tau[j] = tau;
        if (!FIRST) sm.scl[j] = s;
    }
    jprev = j;
}

// Column steps j = 16 TJ .. 16 TJ + 15 (< n), two at a time so that the
// current and next column buffers swap roles without copies.
template <int NS, int RPT, int TJ, bool FIRST, int W>
__device__ __forceinline__ void qr_steps(double (&c)[RPT][NS], const int n, FactorSmemT<W> &sm,
                                         const bool want_t, StepState<NS, RPT> &ss) {
#pragma unroll 1
    for (int q = 0; q < 16; q += 2) {
        const int j = TJ * 16 + q;
        if (j >= n) return;
        one_step<NS, RPT, TJ, FIRST>(j, q, c, n, sm, want_t, ss.xa, ss.xb, ss.rnew, ss.jprev);
        if (j + 1 >= n) return;
        one_step<NS, RPT, TJ, FIRST>(j + 1, q + 1, c, n, sm, want_t, ss.xb, ss.xa, ss.rnew, ss.jprev);
    }
}

// Slot TJ's steps, after part TJ of the previous chunk's staged reflectors
// (if any) has been sent to memory.
template <int NS, int RPT, int TJ, bool FIRST, int W>
__device__ __forceinline__ void qr_slot(double (&c)[RPT][NS], const int n, FactorSmemT<W> &sm,
                                        const bool want_t, StepState<NS, RPT> &ss, const Drain dr) {
    if constexpr (NS == 4 && W == kWaves) {
        if (dr.dst != nullptr) drain_part(dr, TJ);
    }
    qr_steps<NS, RPT, TJ, FIRST>(c, n, sm, want_t, ss);
}

template <int NS, int RPT, bool FIRST, int W, int... TJ>
__device__ __forceinline__ void qr_all_steps(std::integer_sequence<int, TJ...>,
                                             double (&c)[RPT][NS], const int n, FactorSmemT<W> &sm,
                                             const bool want_t, StepState<NS, RPT> &ss, const Drain dr) {
    (qr_slot<NS, RPT, TJ, FIRST>(c, n, sm, want_t, ss, dr), ...);
}

// Householder QR of [R; C] (FIRST == false) or of C alone (FIRST == true,
// rows 0..n-1 of C become R).  On exit c holds the reflector tails V (zeros
// on and above the diagonal of a first chunk, whose unit diagonal is
// implicit), sm.R the updated triangle and, if want_t, the upper triangle
// of sm.T the chunk's T.
template <int NS, int RPT, bool FIRST, int W>
__device__ __forceinline__ void chunk_qr(double (&c)[RPT][NS], const int n,
                                         FactorSmemT<W> &sm, const bool want_t,
                                         const Drain dr = Drain{nullptr, nullptr, 0, 0}) {
    const int tid = step_tid<NS>();
    const int w = tid >> 6, lane = tid & 63, cg = lane & 15, rg = lane >> 4;
    const int rgw = w * 4 + rg;
    StepState<NS, RPT> ss;
#pragma unroll
    for (int i = 0; i < RPT; ++i) ss.xa[i] = __shfl(c[i][0], rg << 4);
    qr_all_steps<NS, RPT, FIRST, W>(std::make_integer_sequence<int, NS>{}, c, n, sm, want_t, ss, dr);
    __syncthreads();
    if (ss.jprev >= 0 && rgw == 0) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 16 * t;
            if (k >= ss.jprev) sm.R[ss.jprev * kLdsStride + k] = ss.rnew[t];
        }
    }
    if constexpr (!FIRST) {
        // reflector tails v_k = s_k x_k (the steps left them unscaled)
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = cg + 16 * t;
            const double sk = (k < n) ? sm.scl[k] : 1.0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) c[i][t] = sk * c[i][t];
        }
    }
}

// Thread rows: row group rgw owns the RPT consecutive rows RPT rgw .. RPT rgw
// + RPT - 1 of a chunk, so a lane moves whole 16-byte pieces (and, over its
// loop, whole cache lines) of each column.  Vector accesses need a 16-byte
// aligned column start; otherwise the same rows go element by element.

template <typename T>
__device__ __forceinline__ bool rows_aligned(const T *p, int64_t ld) {
    return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && (ld * (int64_t)sizeof(T)) % 16 == 0;
}

// Loads rows [0, valid) x columns [0, n) of a chunk at src (ld) into c
// (zeros elsewhere).
template <int NS, int RPT, int W = kWaves>
__device__ __forceinline__ void load_chunk(double (&c)[RPT][NS],
                                           const double *__restrict__ src, int64_t ld, int64_t valid,
                                           int n) {
    const int tid = step_tid<NS>(), w = tid >> 6, lane = tid & 63, cg = lane & 15, rg = lane >> 4;
    const int rgw = w * 4 + rg;
    const bool full = valid >= (int64_t)RPT * 4 * W;
    const bool vec = full && (RPT % 2 == 0) && rows_aligned(src, ld);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int k = cg + 16 * t;
        const double *p = src + (int64_t)rgw * RPT + (int64_t)k * ld;
        if (k < n && vec) {
            // ordinary loads: non-temporal ones streamed this pattern at
            // about a third of the rate (1.35 against 3.6 TB/s, measured)
#pragma unroll
            for (int i = 0; i < RPT; i += 2) {
                const dv2 v = *reinterpret_cast<const dv2 *>(p + i);
                c[i][t] = v.x;
                c[i + 1][t] = v.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                c[i][t] = (k < n && (int64_t)rgw * RPT + i < valid) ? p[i] : 0.0;
        }
    }
}

// Loads of a full chunk (all RPT * 16 rows valid) with no branch around
// them, so that they can stay in flight across other work: the compiler
// keeps a load's result where the chunk lives only if no join follows it.
// A column past n reads column 0 instead; clear_pad_cols zeroes it once the
// data is there.  live == false: a placeholder whose values are never used
// (every lane reads the 16 bytes at src), keeping the loop free of a branch
// around the loads.  VEC: 16-byte pieces (rows_aligned(src, ld) must hold).
template <int NS, int RPT, bool VEC>
__device__ __forceinline__ void issue_full_chunk(double (&c)[RPT][NS], const double *__restrict__ src,
                                                 int64_t ld, int n, bool live = true) {
    const int tid = step_tid<NS>(), w = tid >> 6, lane = tid & 63, cg = lane & 15, rg = lane >> 4;
    const int rgw = w * 4 + rg;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int k = cg + 16 * t;
        const int64_t off = (int64_t)rgw * RPT + (int64_t)(k < n ? k : 0) * ld;
        const double *p = src + (live ? off : 0);
        if constexpr (VEC) {
#pragma unroll
            for (int i = 0; i < RPT; i += 2) {
                const dv2 v = *reinterpret_cast<const dv2 *>(p + i);
                c[i][t] = v.x;
                c[i + 1][t] = v.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < RPT; ++i) c[i][t] = p[i];
        }
    }
}

template <int NS, int RPT>
__device__ __forceinline__ void clear_pad_cols(double (&c)[RPT][NS], int n) {
    if (n >= 16 * NS) return;
    const int cg = step_tid<NS>() & 15;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const bool pad = cg + 16 * t >= n;
#pragma unroll
        for (int i = 0; i < RPT; ++i) c[i][t] = pad ? 0.0 : c[i][t];
    }
}

template <int NS, int RPT, typename OT = double, int W = kWaves>
__device__ __forceinline__ void store_chunk(const double (&c)[RPT][NS],
                                            OT *__restrict__ dst, int64_t ld, int64_t valid, int n,
                                            int t_end = NS) {
    const int tid = step_tid<NS>(), w = tid >> 6, lane = tid & 63, cg = lane & 15, rg = lane >> 4;
    const int rgw = w * 4 + rg;
    const bool full = valid >= (int64_t)RPT * 4 * W;
    constexpr int VW = 16 / sizeof(OT);   // elements per 16-byte store
    const bool vec = full && (RPT % VW == 0) && rows_aligned(dst, ld);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int k = cg + 16 * t;
        OT *p = dst + (int64_t)rgw * RPT + (int64_t)k * ld;
        if (t < t_end && k < n && vec) {
            if constexpr (VW == 2) {
#pragma unroll
                for (int i = 0; i < RPT; i += 2) {
                    double2 v;
                    v.x = c[i][t];
                    v.y = c[i + 1][t];
                    *reinterpret_cast<double2 *>(p + i) = v;
                }
            } else {
#pragma unroll
                for (int i = 0; i < RPT; i += 4) {
                    float4 v;
                    v.x = float(c[i][t]);
                    v.y = float(c[i + 1][t]);
                    v.z = float(c[i + 2][t]);
                    v.w = float(c[i + 3][t]);
                    *reinterpret_cast<float4 *>(p + i) = v;
                }
            }
        } else if (t < t_end && k < n) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if ((int64_t)rgw * RPT + i < valid) p[i] = OT(c[i][t]);
        }
    }
}

// Leaf QR of domain `dom` (step 2): the chunks of the domain in order, a
// geqrt of the first and a tpqrt of [R; chunk] for each later one.
// VT: element type of the stored reflectors (double, or float in the mixed
// mode, where they only feed the FP32 matrix-core applies).  VEC: the
// columns of A allow 16-byte loads (rows_aligned).
//
// The loads of chunk c + 1 are issued as soon as chunk c's reflectors are
// stored and stay in flight while chunk c's T is built and stored, so the
// HBM time of both hides behind that work.  Only the last domain can end in
// a partial chunk; it is loaded with masking at the top of its own
// iteration (the prefetch before it, like the one after the last chunk, is
// a placeholder that reads 16 bytes).  STAGE (wide FP64 kernel, `stage` =
// kStageBytes of LDS): half of each full chunk's reflectors are sent to
// memory during the next chunk's column steps (see Drain).
template <int NS, typename VT, bool VEC, bool STAGE = false, int W>
__device__ __forceinline__ void leaf_domain(FactorSmemT<W> &sm, const double *__restrict__ A, int64_t lda,
                                            VT *__restrict__ V, int64_t ldv, double *__restrict__ Tc,
                                            double *__restrict__ Rdom, const PanelArgs &pa, int keep_q,
                                            int64_t dom, double *stage = nullptr) {
    constexpr int ROWS = chunk_rows(NS);
    constexpr int RPT = rows_per_thread(NS);
    static_assert(ROWS == 4 * W * RPT, "workgroup shape");
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nfull = nrows / ROWS;          // full chunks
    const int64_t tail = nrows - nfull * ROWS;   // rows of a partial last chunk
    const int n = pa.n;
    const int64_t nn = (int64_t)n * n;
    const bool want_t = keep_q != 0;
    // keep_q == 2: each chunk's Gram entries and tau go to its T slot and
    // k_chunk_t builds the T factors after the leaf, off the chunk loop
    const bool defer_t = keep_q == 2;
    auto chunk_t_out = [&](double *dst) {
        if (defer_t) {
            store_gram(sm, dst, n);
        } else {
            build_t(sm, n);
            store_tri(sm.T, dst, n);
        }
    };
    zero_lds(sm.R);
    zero_lds(sm.T);
    __syncthreads();
    double c[RPT][NS];
    if (nfull == 0) {
        // a domain shorter than one chunk
        load_chunk<NS, RPT, W>(c, A + row0, lda, tail, n);
        chunk_qr<NS, RPT, true>(c, n, sm, want_t);
        if (want_t) {
            store_chunk<NS, RPT, VT, W>(c, V + row0, ldv, tail, n);
            chunk_t_out(Tc + dom_chunk0(pa, dom) * nn);
        }
        __syncthreads();
    } else {
        const int64_t nch = nfull + (tail > 0 ? 1 : 0);
        bool staging = false;
        if constexpr (STAGE) staging = want_t && rows_aligned(V + row0, ldv);
        double *pend = nullptr;   // V of the chunk whose slots 2 and 3 sit in the stage
        issue_full_chunk<NS, RPT, VEC>(c, A + row0, lda, n);
        for (int64_t ch = 0; ch < nch; ++ch) {
            const int64_t r0 = row0 + ch * ROWS;
            if (ch == nfull) load_chunk<NS, RPT, W>(c, A + r0, lda, tail, n);
            else clear_pad_cols<NS, RPT>(c, n);
            Drain dr{stage, nullptr, ldv, n};
            if constexpr (STAGE) dr.dst = pend;
            if (ch == 0) chunk_qr<NS, RPT, true>(c, n, sm, want_t, dr);
            else chunk_qr<NS, RPT, false>(c, n, sm, want_t, dr);
            if (want_t) {
                bool staged = false;
                if constexpr (STAGE) {
                    if (staging && ch < nfull) {
                        store_chunk<NS, RPT, VT, W>(c, V + r0, ldv, ROWS, n, 2);   // slots 0 and 1
                        stage_slots(stage, c);
                        pend = V + r0;
                        staged = true;
                    } else {
                        pend = nullptr;
                    }
                }
                if (!staged) store_chunk<NS, RPT, VT, W>(c, V + r0, ldv, ch < nfull ? (int64_t)ROWS : tail, n);
            }
            const bool more = ch + 1 < nfull;
            issue_full_chunk<NS, RPT, VEC>(c, A + row0 + (more ? ch + 1 : 0) * ROWS, lda, n, more);
            if (want_t) chunk_t_out(Tc + (dom_chunk0(pa, dom) + ch) * nn);
            __syncthreads();
        }
        if constexpr (STAGE) {
            if (pend != nullptr)
                for (int part = 0; part < 4; ++part) drain_part(Drain{stage, pend, ldv, n}, part);
        }
    }
    store_tri(sm.R, Rdom + dom * nn, n);
}

// Narrow panels (NS <= 2) fit two workgroups per CU (registers and LDS), which
// hides step latency whenever there are more domains than CUs.
template <int NS>
constexpr int leaf_min_blocks() { return NS == 2 ? 2 : 1; }
template <int NS>
constexpr int leaf_threads() { return kFactorThreads; }

// The wide FP64 leaf stages half of each chunk's reflectors in LDS.
template <int NS, typename VT>
constexpr bool leaf_stages() { return NS == 4 && std::is_same<VT, double>::value; }

template <int NS>
using LeafSmem = FactorSmem;

template <int NS, typename VT, bool VEC>
__global__ __launch_bounds__(leaf_threads<NS>(), leaf_min_blocks<NS>()) void k_leaf(const double *__restrict__ A, int64_t lda,
                                                 VT *__restrict__ V, int64_t ldv,
                                                 double *__restrict__ Tc, double *__restrict__ Rdom,
                                                 PanelArgs pa, int keep_q) {
    extern __shared__ double smem_raw[];
    LeafSmem<NS> &sm = *reinterpret_cast<LeafSmem<NS> *>(smem_raw);
    constexpr bool S = leaf_stages<NS, VT>();
    leaf_domain<NS, VT, VEC, S>(sm, A, lda, V, ldv, Tc, Rdom, pa, keep_q, blockIdx.x,
                                S ? smem_raw + sizeof(LeafSmem<NS>) / sizeof(double) : nullptr);
}

// T of every chunk of the panel (the leaf left each chunk's Gram entries and
// tau in its slot: keep_q == 2), slots 0 .. total - 1.  Workgroup b takes
// slots b, b + gridDim.x, ...; the next slot's entries are loaded into
// registers while the current T is built, so each slot costs one memory
// round trip less than a workgroup per slot.
__global__ __launch_bounds__(kFactorThreads) void k_chunk_t(double *__restrict__ Tc, int64_t total, int n) {
    extern __shared__ double smem_raw[];
    TBuildSmem &sm = *reinterpret_cast<TBuildSmem *>(smem_raw);
    const int64_t nn = (int64_t)n * n;
    constexpr int kPer = 64 * 64 / kFactorThreads;
    if (n % 16 != 0) {
        // build_t's block products read Gram entries of the last 16-column
        // block past n (times zero); nothing below writes them
        for (int e = threadIdx.x; e < 64 * kLdsStride; e += kFactorThreads) sm.T[e] = 0.0;
    }
    double gv[kPer];
    auto fetch = [&](int64_t g) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = threadIdx.x + kFactorThreads * u;
            gv[u] = (e < n * n) ? Tc[g * nn + e] : 0.0;
        }
    };
    int64_t g = blockIdx.x;
    if (g < total) fetch(g);
    for (; g < total; g += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = threadIdx.x + kFactorThreads * u;
            if (e < n * n) {
                const int r = e % n, c = e / n;
                if (r > c) sm.T[r * kLdsStride + c] = gv[u];
                else if (r == c) sm.tau[r] = gv[u];
            }
        }
        const int64_t next = g + gridDim.x;
        if (next < total) fetch(next);
        __syncthreads();
        build_t(sm, n);
        store_tri(sm.T, Tc + g * nn, n);
    }
}

// ---- batched forms: grid.y walks the matrix list, grid.x the domains /
// chains of the listed matrix (a workgroup past its matrix's count returns).
template <int NS>
__global__ __launch_bounds__(leaf_threads<NS>(), leaf_min_blocks<NS>()) void k_leaf_b(const BMat *__restrict__ mats,
                                                   const int *__restrict__ list) {
    extern __shared__ double smem_raw[];
    LeafSmem<NS> &sm = *reinterpret_cast<LeafSmem<NS> *>(smem_raw);
    const BMat &M = mats[list[blockIdx.y]];
    const int64_t dom = blockIdx.x;
    if (dom >= M.pa.P) return;
    const bool vec = rows_aligned(M.A, M.lda) && (M.pa.mb % 2) == 0;
    if (M.prec) {
        if (vec) leaf_domain<NS, float, true>(sm, M.A, M.lda, M.V32, M.pa.m, M.Tc, M.Rdom, M.pa, 1, dom);
        else leaf_domain<NS, float, false>(sm, M.A, M.lda, M.V32, M.pa.m, M.Tc, M.Rdom, M.pa, 1, dom);
    } else {
        if (vec) leaf_domain<NS, double, true>(sm, M.A, M.lda, M.V, M.pa.m, M.Tc, M.Rdom, M.pa, 1, dom);
        else leaf_domain<NS, double, false>(sm, M.A, M.lda, M.V, M.pa.m, M.Tc, M.Rdom, M.pa, 1, dom);
    }
}

template <int NS>
static hipError_t launch_leaf_b_ns(const BMat *mats, const int *list, int cnt, int64_t gx, hipStream_t st) {
    const size_t sh = sizeof(LeafSmem<NS>);
    hipError_t e = hipFuncSetAttribute((const void *)k_leaf_b<NS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("batch_leaf_factor", st);
    hipLaunchKernelGGL(k_leaf_b<NS>, dim3((unsigned)gx, (unsigned)cnt), dim3(leaf_threads<NS>()), sh, st, mats,
                       list);
    return hipGetLastError();
}

hipError_t launch_leaf_b(const BMat *mats, const int *list, int cnt, int64_t gx, int ns, hipStream_t st) {
    if (cnt <= 0 || gx <= 0) return hipSuccess;
    switch (ns) {
        case 1: return launch_leaf_b_ns<1>(mats, list, cnt, gx, st);
        case 2: return launch_leaf_b_ns<2>(mats, list, cnt, gx, st);
        default: return launch_leaf_b_ns<4>(mats, list, cnt, gx, st);
    }
}

template <int NS, typename VT, bool VEC>
static hipError_t launch_leaf_nsv(const double *A, int64_t lda, VT *V, int64_t ldv, double *Tc,
                                  double *Rdom, const PanelArgs &pa, int keep_q, const char *tag,
                                  hipStream_t st) {
    const size_t sh = sizeof(LeafSmem<NS>) + (leaf_stages<NS, VT>() ? kStageBytes : 0);
    hipError_t e = hipFuncSetAttribute((const void *)k_leaf<NS, VT, VEC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps(tag, st);
    hipLaunchKernelGGL((k_leaf<NS, VT, VEC>), dim3((unsigned)pa.P), dim3(leaf_threads<NS>()), sh, st, A, lda, V,
                       ldv, Tc, Rdom, pa, keep_q);
    return hipGetLastError();
}

template <int NS, typename VT>
static hipError_t launch_leaf_ns(const double *A, int64_t lda, VT *V, int64_t ldv, double *Tc,
                                 double *Rdom, const PanelArgs &pa, int keep_q, const char *tag,
                                 hipStream_t st) {
    // 16-byte loads need every chunk's first row 16-byte aligned: A itself,
    // every column start (lda) and every domain start (mb) must be even
    const bool vec = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda * (int64_t)sizeof(double)) % 16 == 0 &&
                     (pa.mb % 2) == 0;
    return vec ? launch_leaf_nsv<NS, VT, true>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, tag, st)
               : launch_leaf_nsv<NS, VT, false>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, tag, st);
}

template <typename VT>
static hipError_t launch_leaf_t(const double *A, int64_t lda, VT *V, int64_t ldv, double *Tc, double *Rdom,
                                const PanelArgs &pa, int keep_q, const char *tag, hipStream_t st) {
    switch (pa.ns) {
        case 1: return launch_leaf_ns<1, VT>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, tag, st);
        case 2: return launch_leaf_ns<2, VT>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, tag, st);
        default: return launch_leaf_ns<4, VT>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, tag, st);
    }
}

hipError_t launch_chunk_t(double *Tc, const PanelArgs &pa, int64_t total_chunks, hipStream_t st) {
    if (total_chunks <= 0) return hipSuccess;
    const size_t sh = sizeof(TBuildSmem);
    hipError_t e = hipFuncSetAttribute((const void *)k_chunk_t, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    ProfScope ps("chunk_t", st);
    // two workgroups per CU (the LDS fits two)
    const int64_t grid = total_chunks < 512 ? total_chunks : 512;
    hipLaunchKernelGGL(k_chunk_t, dim3((unsigned)grid), dim3(kFactorThreads), sh, st, Tc, total_chunks, pa.n);
    return hipGetLastError();
}

hipError_t launch_leaf(const double *A, int64_t lda, double *V, int64_t ldv, double *Tc, double *Rdom,
                       const PanelArgs &pa, int keep_q, hipStream_t st) {
    return launch_leaf_t<double>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, "leaf_factor", st);
}

hipError_t launch_leaf32(const double *A, int64_t lda, float *V, int64_t ldv, double *Tc, double *Rdom,
                         const PanelArgs &pa, int keep_q, hipStream_t st) {
    return launch_leaf_t<float>(A, lda, V, ldv, Tc, Rdom, pa, keep_q, "leaf_factor_v32", st);
}

}  // namespace tsqr
