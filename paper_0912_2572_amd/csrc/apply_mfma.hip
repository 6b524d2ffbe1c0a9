// apply_mfma.hip -- leaf part of Q^T B / Q B on matrix cores, for blocks of
// up to 16 columns of B (least squares, refinement corrections, and the
// trailing update between 64-column panels).
//
// Per chunk of a domain (compact-WY factor I - Y T Y^T, Sec. 2.2):
//     W = Yb + V^T B_c          (Yb = the domain's top n rows; 0 on a first
//                                chunk, whose V has an implicit unit diagonal)
//     Z = T^T W  (Q^T)  or  T W  (Q)
//     Yb -= Z,   B_c -= V Z
// W is reduced over the chunk's rows by 16x16x4 MFMA tiles with the row index
// as the reduction dimension (each wave takes a quarter of the rows, the
// four partials meet in LDS); the update runs transposed,
// (B_c - V Z)^T = B_c^T - Z^T V^T, so that each store writes 16 consecutive
// rows of a column.
//
// Two precisions share the code: FP64 (V in FP64, v_mfma_f64_16x16x4f64) and
// the mixed mode's FP32 path (V stored in FP32, v_mfma_f32_16x16x4f32 with
// FP32 accumulation, W and Z in FP32).  B and the running top rows Yb stay
// FP64, and B is updated as B - (V Z) with only the product in the tile
// precision, so an FP32 apply perturbs B by about u32 times the size of the
// update rather than u32 times |B|.
#include "common.h"
#include "kernels.h"
#include "mfma.h"
#include "prof.h"

namespace tsqr {

constexpr int KBM = 16;   // columns of B per workgroup

template <typename Tile>
struct ApplyMSmem {
    using T = typename Tile::T;
    T Tm[64 * kLdsStride];
    T Wp[4][64][KBM];   // per-wave partials of W; then W in Wp[1] and Z in Wp[0]
    double Y[64][KBM];  // the domain's top n rows of B (columns of this block)
};
static_assert(2 * sizeof(ApplyMSmem<TileF64>) <= 160 * 1024, "two workgroups per CU");

// V element of a chunk with the implicit unit diagonal of a first chunk.
template <typename VT>
__device__ __forceinline__ VT v_elem(const VT *__restrict__ Vc, int64_t ldv, int64_t row, int col,
                                     int64_t valid, int n, bool first) {
    if (row >= valid || col >= n) return VT(0);
    if (first && row <= col) return (row == col) ? VT(1) : VT(0);
    return Vc[row + (int64_t)col * ldv];
}

// Four consecutive entries p[0..3] as 16-byte loads (p 16-byte aligned),
// or zeros when !ok; FP64 reads two double2, FP32 one float4, and the
// entries are converted to T.
template <typename T, typename S>
__device__ __forceinline__ void load4(const S *__restrict__ p, bool ok, T (&v)[4]) {
    if constexpr (sizeof(S) == 8) {
        double2 x0 = {0.0, 0.0}, x1 = {0.0, 0.0};
        if (ok) {
            x0 = reinterpret_cast<const double2 *>(p)[0];
            x1 = reinterpret_cast<const double2 *>(p)[1];
        }
        v[0] = T(x0.x); v[1] = T(x0.y); v[2] = T(x1.x); v[3] = T(x1.y);
    } else {
        float4 x = {0.f, 0.f, 0.f, 0.f};
        if (ok) x = *reinterpret_cast<const float4 *>(p);
        v[0] = T(x.x); v[1] = T(x.y); v[2] = T(x.z); v[3] = T(x.w);
    }
}

// A wave's row range [r, r + rows) of V and B can be read 4 rows at a time
// with 16-byte loads: whole 16-row blocks, every column start 16-byte aligned.
template <typename VT>
__device__ __forceinline__ bool wide_rows_ok(const VT *v, int64_t ldv, const double *b, int64_t ldb, int64_t rows) {
    return rows > 0 && rows % 16 == 0 && (reinterpret_cast<uintptr_t>(v) & 15) == 0 &&
           (reinterpret_cast<uintptr_t>(b) & 15) == 0 && (ldv * (int64_t)sizeof(VT)) % 16 == 0 &&
           (ldb * 8) % 16 == 0;
}

template <typename Tile>
__device__ __forceinline__ void chunk_apply_m(ApplyMSmem<Tile> &sm, const typename Tile::T *__restrict__ Vc, int64_t ldv,
                              const double *__restrict__ Tk, const double *__restrict__ Bin, int64_t ldbi,
                              double *__restrict__ Bout, int64_t ldbo, int64_t valid, int n, int kc,
                              bool first, int trans) {
    using T = typename Tile::T;
    using Acc = typename Tile::Acc;
    const int tid = local_tid(), lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int mtn = (n + 15) >> 4;             // 16-reflector tiles
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, q = e >> 6;
        sm.Tm[r * kLdsStride + q] = (r < n && q < n) ? T(Tk[r + (int64_t)q * n]) : T(0);
    }
    // W partial over this wave's rows: W[m][j] += sum_r V[r][m] B[r][j]
    {
        Acc acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = Acc{0, 0, 0, 0};
        const int64_t per = ((valid + 15) / 16 + 3) / 4 * 16;   // rows per wave, multiple of 16
        const int64_t lo = w * per, hi = (lo + per < valid) ? lo + per : valid;
        if (!first && wide_rows_ok(Vc + lo, ldv, Bin + lo, ldbi, hi - lo)) {
            // 16-byte loads of 4 consecutive rows per lane (as in the first pass)
#pragma unroll 1
            for (int64_t r16 = lo; r16 < hi; r16 += 16) {
                const int64_t rb = r16 + 4 * l4;
                T b4[4];
                load4<T>(Bin + rb + (int64_t)l16 * ldbi, l16 < kc, b4);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    if (mt >= mtn) break;
                    T a4[4];
                    load4<T>(Vc + rb + (int64_t)(16 * mt + l16) * ldv, 16 * mt + l16 < n, a4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[mt] = Tile::mfma(a4[q], b4[q], acc[mt]);
                }
            }
        } else {
            for (int64_t r4 = lo; r4 < hi; r4 += 4) {
                const int64_t row = r4 + l4;
                double bv = 0.0;
                if (row < hi && l16 < kc) {
                    if (first && !trans && row < n) bv = sm.Y[row][l16];
                    else bv = Bin[row + (int64_t)l16 * ldbi];
                }
                const T b = T(bv);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    if (mt >= mtn) break;
                    const T a = (row < hi) ? v_elem<T>(Vc, ldv, row, 16 * mt + l16, valid, n, first) : T(0);
                    acc[mt] = Tile::mfma(a, b, acc[mt]);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Wp[w][16 * mt + Tile::drow(r, lane)][l16] = acc[mt][r];
    }
    __syncthreads();
    for (int e = tid; e < 64 * KBM; e += 256) {
        const int m = e >> 4, j = e & 15;
        T s = ((sm.Wp[0][m][j] + sm.Wp[1][m][j]) + sm.Wp[2][m][j]) + sm.Wp[3][m][j];
        if (!first) s += T(sm.Y[m][j]);
        sm.Wp[1][m][j] = s;   // W: each entry read and written by one thread
    }
    __syncthreads();
    // Z = op(T) W (W in Wp[1]) on the matrix cores, written over the
    // partial buffer of wave 0: wave w computes rows 16 w .. 16 w + 15 (T is
    // zero outside its upper triangle and past n, so the full 64-wide sum is
    // op(T) W; W rows past n are not formed and enter as zeros)
    {
        Acc acc = Acc{0, 0, 0, 0};
        const int i = 16 * w + l16;
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
            if (4 * kb >= n) break;
            const int q = 4 * kb + l4;
            const T a = trans ? sm.Tm[q * kLdsStride + i] : sm.Tm[i * kLdsStride + q];
            const T b = (q < n) ? sm.Wp[1][q][l16] : T(0);
            acc = Tile::mfma(a, b, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.Wp[0][16 * w + Tile::drow(r, lane)][l16] = acc[r];
    }
    __syncthreads();
    if (!first)
        for (int e = tid; e < 64 * KBM; e += 256) {
            const int i = e >> 4, j = e & 15;
            sm.Y[i][j] -= (double)sm.Wp[0][i][j];
        }
    // B_c^T -= Z^T V^T over 16-row tiles: wave w takes tiles w, w + 4, ...
    const int kbn = (n + 3) >> 2;
    for (int64_t t0 = 16 * w; t0 < valid; t0 += 64) {
        const int64_t row = t0 + l16;
        T vv[16];
#pragma unroll
        for (int kb = 0; kb < 16; ++kb)
            vv[kb] = (kb < kbn) ? v_elem<T>(Vc, ldv, row, 4 * kb + l4, valid, n, first) : T(0);
        double b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = Tile::drow(r, lane);
            b[r] = 0.0;
            if (row < valid && col < kc) {
                if (first && !trans && row < n) b[r] = sm.Y[row][col];
                else b[r] = Bin[row + (int64_t)col * ldbi];
            }
        }
        Acc acc = Acc{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
            if (kb >= kbn) break;
            acc = Tile::mfma(sm.Wp[0][4 * kb + l4][l16], vv[kb], acc);   // Z^T[col][refl] V^T
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = Tile::drow(r, lane);
            if (row < valid && col < kc) {
                const double out = b[r] - (double)acc[r];
                if (first && trans && row < n) sm.Y[row][col] = out;
                else Bout[row + (int64_t)col * ldbo] = out;
            }
        }
    }
    __syncthreads();
}

// Leaf part for domain `dom` and the 16-column block `cblk` of B.
template <typename Tile>
__device__ __forceinline__ void leaf_apply_domain(ApplyMSmem<Tile> &sm, const typename Tile::T *__restrict__ V,
                                                  int64_t ldv, const double *__restrict__ Tc,
                                                  const PanelArgs &pa, const double *__restrict__ Bsrc,
                                                  int64_t ldbs, double *__restrict__ B, int64_t ldb, int64_t k,
                                                  int trans, int64_t dom, int64_t cblk) {
    const int64_t c0 = cblk * KBM;
    const int kc = (int)((k - c0 < KBM) ? k - c0 : KBM);
    const int n = pa.n;
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    const int64_t nn = (int64_t)n * n;
    const double *Bs0 = Bsrc + c0 * ldbs;
    double *B0 = B + c0 * ldb;
    const int tid = threadIdx.x;
    if (trans) {
        for (int64_t ch = 0; ch < nch; ++ch) {
            const int64_t r0 = row0 + ch * pa.chunk;
            const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
            chunk_apply_m<Tile>(sm, V + r0, ldv, Tc + (dom_chunk0(pa, dom) + ch) * nn, Bs0 + r0, ldbs, B0 + r0,
                                ldb, valid, n, kc, ch == 0, 1);
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
            chunk_apply_m<Tile>(sm, V + r0, ldv, Tc + (dom_chunk0(pa, dom) + ch) * nn, Bs0 + r0, ldbs, B0 + r0,
                                ldb, valid, n, kc, ch == 0, 0);
        }
    }
}

// Workgroup order: groups of 8 domains x ncb column blocks, the column
// blocks of one domain 8 workgroups apart.  Workgroups go to the 8 XCDs
// round-robin by index, so a domain's column blocks share one XCD (one L2)
// and run side by side: its V comes from HBM about once instead of ncb times.
template <typename Tile>
__global__ __launch_bounds__(256) void k_leaf_apply_m(const typename Tile::T *__restrict__ V, int64_t ldv,
                                                      const double *__restrict__ Tc, PanelArgs pa,
                                                      const double *__restrict__ Bsrc, int64_t ldbs,
                                                      double *__restrict__ B, int64_t ldb, int64_t k,
                                                      int trans, int ncb) {
    extern __shared__ double smem_raw[];
    ApplyMSmem<Tile> &sm = *reinterpret_cast<ApplyMSmem<Tile> *>(smem_raw);
    const int64_t b = blockIdx.x, per = 8 * (int64_t)ncb;
    const int64_t within = b % per;
    const int64_t dom = (b / per) * 8 + within % 8;
    const int64_t cblk = within / 8;
    if (dom >= pa.P) return;
    leaf_apply_domain<Tile>(sm, V, ldv, Tc, pa, Bsrc, ldbs, B, ldb, k, trans, dom, cblk);
}

template <typename Tile>
static hipError_t launch_apply_m(const typename Tile::T *V, int64_t ldv, const double *Tc,
                                 const PanelArgs &pa, const double *Bsrc, int64_t ldbs, double *B,
                                 int64_t ldb, int64_t k, int trans, const char *tag, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const size_t sh = sizeof(ApplyMSmem<Tile>);
    hipError_t e = hipFuncSetAttribute((const void *)k_leaf_apply_m<Tile>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    const int ncb = (int)((k + KBM - 1) / KBM);
    const int64_t groups = (pa.P + 7) / 8;
    ProfScope ps(tag, st);
    hipLaunchKernelGGL(k_leaf_apply_m<Tile>, dim3((unsigned)(groups * 8 * ncb)), dim3(256), sh, st, V, ldv, Tc,
                       pa, Bsrc, ldbs, B, ldb, k, trans, ncb);
    return hipGetLastError();
}

hipError_t launch_leaf_apply_m(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                               const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                               int trans, hipStream_t st) {
    return launch_apply_m<TileF64>(V, ldv, Tc, pa, Bsrc, ldbs, B, ldb, k, trans,
                                   trans ? "leaf_apply_qt" : "leaf_apply_q", st);
}

hipError_t launch_leaf_apply_m32(const float *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                                 const double *Bsrc, int64_t ldbs, double *B, int64_t ldb, int64_t k,
                                 int trans, hipStream_t st) {
    return launch_apply_m<TileF32>(V, ldv, Tc, pa, Bsrc, ldbs, B, ldb, k, trans,
                                   trans ? "leaf_apply_qt_f32" : "leaf_apply_q_f32", st);
}

// ---------------------------------------------------------------------------
// Three-pass leaf apply for few columns (k <= 16).  The chunk chain of a
// domain couples chunks only through the n x k running top rows Y, so
//   pass 1 (every chunk at once):  P_c = V_c^T B_c            (a first chunk
//                                  from row n on: its top rows are Y)
//   pass 2 (one workgroup/domain): the chain on n x k blocks,
//          Q^T: W_0 = V_0top^T Y + P_0, Z_0 = T_0^T W_0, Y <- Y - V_0top Z_0,
//               then W_c = Y + P_c, Z_c = T_c^T W_c, Y <- Y - Z_c (c = 1..),
//          Q:   chunks last to first with T_c, chunk 0 last, top rows
//               written as Y - V_0top Z_0;
//   pass 3 (every chunk at once):  B_c <- B_c - V_c Z_c   (rows below the
//                                  top rows of a first chunk).
// V is streamed twice across the whole device instead of once chunk after
// chunk; the chain touches only T and n x k blocks.  P_c and Z_c are n x k
// column-major blocks, one per chunk.

// Rows [rlo, valid) of chunk c: W(n x kc) = V_c^T B_c, one partial per wave
// in sm.Wp (tile precision); the caller adds the four in wave order.
template <typename Tile>
struct VtbSmem {
    using T = typename Tile::T;
    // per-wave partials of V^T B, entry (wave w, row m, column j < kc) at
    // (64 w + m) kc + j: a launch sizes the LDS by its own kc (vtb_lds_bytes)
    T Wp[4 * 64 * KBM];
};
template <typename Tile>
constexpr size_t vtb_lds_bytes(int64_t kc) {
    return (size_t)4 * 64 * (size_t)kc * sizeof(typename Tile::T);
}

template <typename Tile>
__device__ __forceinline__ void chunk_vtb(VtbSmem<Tile> &sm, const typename Tile::T *__restrict__ Vc,
                                          int64_t ldv, const double *__restrict__ Bc, int64_t ldb,
                                          int64_t rlo, int64_t valid, int n, int kc, bool first) {
    using T = typename Tile::T;
    using Acc = typename Tile::Acc;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int mtn = (n + 15) >> 4;
    Acc acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = Acc{0, 0, 0, 0};
    const int64_t span = valid - rlo;
    const int64_t per = ((span + 15) / 16 + 3) / 4 * 16;
    const int64_t lo = rlo + w * per, hi = (lo + per < valid) ? lo + per : valid;
    if (wide_rows_ok(Vc + lo, ldv, Bc + lo, ldb, hi - lo)) {
        // each lane reads 4 consecutive rows of its column with 16-byte
        // loads (16 rows x 16 columns per instruction); MFMA q takes row
        // 4 l4 + q of the 16-row block as its k = l4 element
        for (int64_t r16 = lo; r16 < hi; r16 += 16) {
            const int64_t rb = r16 + 4 * l4;
            T b4[4];
            load4<T>(Bc + rb + (int64_t)l16 * ldb, l16 < kc, b4);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                if (mt >= mtn) break;
                T a4[4];
                load4<T>(Vc + rb + (int64_t)(16 * mt + l16) * ldv, 16 * mt + l16 < n, a4);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[mt] = Tile::mfma(a4[q], b4[q], acc[mt]);
            }
        }
    } else {
        for (int64_t r4 = lo; r4 < hi; r4 += 4) {
            const int64_t row = r4 + l4;
            const T b = T((row < hi && l16 < kc) ? Bc[row + (int64_t)l16 * ldb] : 0.0);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                if (mt >= mtn) break;
                const T a = (row < hi) ? v_elem<T>(Vc, ldv, row, 16 * mt + l16, valid, n, first) : T(0);
                acc[mt] = Tile::mfma(a, b, acc[mt]);
            }
        }
    }
    if (l16 < kc) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Wp[(64 * w + 16 * mt + Tile::drow(r, lane)) * kc + l16] = acc[mt][r];
    }
    __syncthreads();
}

template <typename Tile>
__device__ __forceinline__ void apply_p1_body(const typename Tile::T *__restrict__ V, int64_t ldv,
                                              const PanelArgs &pa, const double *__restrict__ B, int64_t ldb,
                                              int64_t k, double *__restrict__ Pc, int64_t dom, int64_t ch) {
    extern __shared__ double smem_raw[];
    VtbSmem<Tile> &sm = *reinterpret_cast<VtbSmem<Tile> *>(smem_raw);
    const int n = pa.n;
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    if (ch >= nch) return;
    const int kc = (int)k;
    const int64_t r0 = row0 + ch * pa.chunk;
    const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
    chunk_vtb<Tile>(sm, V + r0, ldv, B + r0, ldb, ch == 0 ? n : 0, valid, n, kc, ch == 0);
    // P_c = the four waves' partials added in wave order
    using T = typename Tile::T;
    double *P = Pc + (dom_chunk0(pa, dom) + ch) * (int64_t)n * k;
    const int ws = 64 * kc;
    for (int e = threadIdx.x; e < n * kc; e += 256) {
        const int m = e % n, j = e / n, o = m * kc + j;
        const T sum = ((sm.Wp[o] + sm.Wp[ws + o]) + sm.Wp[2 * ws + o]) + sm.Wp[3 * ws + o];
        P[e] = (double)sum;
    }
}

template <typename Tile>
__global__ __launch_bounds__(256) void k_apply_p1(const typename Tile::T *__restrict__ V, int64_t ldv,
                                                  PanelArgs pa, const double *__restrict__ B, int64_t ldb,
                                                  int64_t k, double *__restrict__ Pc) {
    apply_p1_body<Tile>(V, ldv, pa, B, ldb, k, Pc, blockIdx.y, blockIdx.x);
}

struct ChainSmem {
    double Tm[64 * kLdsStride];
    // unit lower V_0top of the first chunk, its lower triangle (diagonal of
    // ones included) packed by rows: entry (r, c), c <= r, at r (r + 1) / 2 + c.
    // Packed, the struct fits two workgroups in a CU's LDS.
    double V0[64 * 65 / 2];
    double Y[64][KBM];
    double W[64][KBM];
    double Z[64][KBM];
};
static_assert(2 * sizeof(ChainSmem) <= 160 * 1024, "two chain workgroups per CU");
__device__ __forceinline__ int v0_at(int r, int c) { return r * (r + 1) / 2 + c; }

// Pass 2 for one domain (FP64).
__device__ __forceinline__ void apply_p2_body(const double *__restrict__ V64, const float *__restrict__ V32,
                                              int64_t ldv, const double *__restrict__ Tc, const PanelArgs &pa,
                                              double *__restrict__ B, int64_t ldb, int64_t k, int trans,
                                              const double *__restrict__ Pc, double *__restrict__ Zc,
                                              int64_t dom) {
    extern __shared__ double smem_raw[];
    ChainSmem &sm = *reinterpret_cast<ChainSmem *>(smem_raw);
    const int n = pa.n, kc = (int)k, tid = threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    for (int e = tid; e < 64 * KBM; e += 256) {
        const int r = e >> 4, c = e & 15;
        sm.Y[r][c] = (r < n && c < kc) ? B[row0 + r + (int64_t)c * ldb] : 0.0;
    }
    // V_0top, unit lower triangular (the reflector storage precision)
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, q = e >> 6;
        if (q > r) continue;
        double v = 0.0;
        if (r < n && q < n) {
            if (r == q) v = 1.0;
            else v = V32 ? (double)V32[row0 + r + (int64_t)q * ldv] : V64[row0 + r + (int64_t)q * ldv];
        }
        sm.V0[v0_at(r, q)] = v;
    }
    // Only the n x kc live entries are computed (e < n kc: i = e % n, j = e / n).
    // The next chunk's T and P_c are fetched into registers while the current
    // chunk is processed (loads retire in order, so a P_c loaded inside the
    // step would also wait for the T fetched ahead).
    const int live = n * kc;
    constexpr int kTPer = 64 * 64 / 256;    // T entries per thread
    constexpr int kPPer = 64 * KBM / 256;   // P_c entries per thread (live <= 64 KBM)
    double tnext[kTPer], pnext[kPPer];
    auto fetch_t = [&](int64_t ch) {
        const double *Tk = Tc + (dom_chunk0(pa, dom) + ch) * nn;
#pragma unroll
        for (int u = 0; u < kTPer; ++u) {
            const int e = tid + 256 * u, r = e & 63, q = e >> 6;
            tnext[u] = (r < n && q < n) ? Tk[r + (int64_t)q * n] : 0.0;
        }
        // P_c is n x kc, column-major with ld n: entry (e % n, e / n) at e
        const double *P = Pc + (dom_chunk0(pa, dom) + ch) * (int64_t)n * k;
#pragma unroll
        for (int u = 0; u < kPPer; ++u) {
            const int e = tid + 256 * u;
            pnext[u] = (e < live) ? P[e] : 0.0;
        }
    };
    auto chunk_step = [&](int64_t ch, int64_t ch_next) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTPer; ++u) {
            const int e = tid + 256 * u, r = e & 63, q = e >> 6;
            sm.Tm[r * kLdsStride + q] = tnext[u];
        }
        double pcur[kPPer];
#pragma unroll
        for (int u = 0; u < kPPer; ++u) pcur[u] = pnext[u];
        if (ch_next >= 0) fetch_t(ch_next);
        // W = (V_0top^T Y on a first chunk, else Y) + P_c
#pragma unroll
        for (int u = 0; u < kPPer; ++u) {
            const int e = tid + 256 * u;
            if (e >= live) continue;
            const int m = e % n, j = e / n;
            double wv = 0.0;
            if (ch == 0) {
                for (int r = m; r < n; ++r) wv = fma(sm.V0[v0_at(r, m)], sm.Y[r][j], wv);
            } else {
                wv = sm.Y[m][j];
            }
            sm.W[m][j] = wv + pcur[u];
        }
        __syncthreads();
        for (int e = tid; e < live; e += 256) {
            const int i = e % n, j = e / n;
            double z = 0.0;
            if (trans) {
                for (int q = 0; q <= i; ++q) z = fma(sm.Tm[q * kLdsStride + i], sm.W[q][j], z);
            } else {
                for (int q = i; q < n; ++q) z = fma(sm.Tm[i * kLdsStride + q], sm.W[q][j], z);
            }
            sm.Z[i][j] = z;
            Zc[(dom_chunk0(pa, dom) + ch) * (int64_t)n * k + i + (int64_t)j * n] = z;
        }
        __syncthreads();
        // Y <- Y - Z, or on a first chunk Y <- Y - V_0top Z
        for (int e = tid; e < live; e += 256) {
            const int i = e % n, j = e / n;
            if (ch == 0) {
                double u = 0.0;
                for (int q = 0; q <= i; ++q) u = fma(sm.V0[v0_at(i, q)], sm.Z[q][j], u);
                sm.W[i][j] = sm.Y[i][j] - u;
            } else {
                sm.Y[i][j] -= sm.Z[i][j];
            }
        }
        if (ch == 0) {
            __syncthreads();
            for (int e = tid; e < live; e += 256) {
                const int i = e % n, j = e / n;
                sm.Y[i][j] = sm.W[i][j];
            }
        }
    };
    if (trans) {
        fetch_t(0);
        for (int64_t ch = 0; ch < nch; ++ch) chunk_step(ch, ch + 1 < nch ? ch + 1 : -1);
    } else {
        fetch_t(nch - 1);
        for (int64_t ch = nch - 1; ch >= 0; --ch) chunk_step(ch, ch - 1);
    }
    __syncthreads();
    for (int e = tid; e < 64 * KBM; e += 256) {
        const int r = e >> 4, c = e & 15;
        if (r < n && c < kc) B[row0 + r + (int64_t)c * ldb] = sm.Y[r][c];
    }
}

__global__ __launch_bounds__(256) void k_apply_p2(const double *__restrict__ V64, const float *__restrict__ V32,
                                                  int64_t ldv, const double *__restrict__ Tc, PanelArgs pa,
                                                  double *__restrict__ B, int64_t ldb, int64_t k, int trans,
                                                  const double *__restrict__ Pc, double *__restrict__ Zc) {
    apply_p2_body(V64, V32, ldv, Tc, pa, B, ldb, k, trans, Pc, Zc, blockIdx.x);
}

// Pass 3: B_c <- B_c - V_c Z_c over the chunk's rows (a first chunk from
// row n on), transposed MFMA form as in chunk_apply_m; the Z operand stays in
// registers, so the kernel needs no LDS and many workgroups share a CU.
template <typename Tile>
__device__ __forceinline__ void apply_p3_body(const typename Tile::T *__restrict__ V, int64_t ldv,
                                              const PanelArgs &pa, double *__restrict__ B, int64_t ldb, int64_t k,
                                              const double *__restrict__ Zc, int64_t dom, int64_t ch) {
    using T = typename Tile::T;
    using Acc = typename Tile::Acc;
    const int n = pa.n, kc = (int)k;
    const int64_t row0 = dom_row0(pa, dom);
    const int64_t nrows = dom_rows(pa, dom);
    const int64_t nch = (nrows + pa.chunk - 1) / pa.chunk;
    if (ch >= nch) return;
    const int64_t r0 = row0 + ch * pa.chunk;
    const int64_t valid = (nrows - ch * pa.chunk < pa.chunk) ? nrows - ch * pa.chunk : pa.chunk;
    const bool first = ch == 0;
    const double *Z = Zc + (dom_chunk0(pa, dom) + ch) * (int64_t)n * k;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int kbn = (n + 3) >> 2;
    // A[i][q] = Z^T[col i][reflector q] for q = 4 kb + l4
    T za[16];
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
        const int q = 4 * kb + l4;
        za[kb] = (q < n && l16 < kc) ? T(Z[q + (int64_t)l16 * n]) : T(0);
    }
    const T *Vc = V + r0;
    double *Bc = B + r0;
    for (int64_t t0 = 16 * w; t0 < valid; t0 += 64) {
        const int64_t row = t0 + l16;
        const bool live = row < valid && !(first && row < n);
        T vv[16];
#pragma unroll
        for (int kb = 0; kb < 16; ++kb)
            vv[kb] = (kb < kbn && live) ? v_elem<T>(Vc, ldv, row, 4 * kb + l4, valid, n, first) : T(0);
        Acc acc = Acc{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
            if (kb >= kbn) break;
            acc = Tile::mfma(za[kb], vv[kb], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = Tile::drow(r, lane);
            if (live && col < kc) Bc[row + (int64_t)col * ldb] -= (double)acc[r];
        }
    }
}

template <typename Tile>
__global__ __launch_bounds__(256) void k_apply_p3(const typename Tile::T *__restrict__ V, int64_t ldv,
                                                  PanelArgs pa, double *__restrict__ B, int64_t ldb, int64_t k,
                                                  const double *__restrict__ Zc) {
    apply_p3_body<Tile>(V, ldv, pa, B, ldb, k, Zc, blockIdx.y, blockIdx.x);
}

// ---- batched forms on each listed matrix's vector F (k = 1); grid.x walks
// the matrix's chunks (pass 1, 3) or domains (pass 2); sweep > 0 skips
// converged matrices.
__device__ __forceinline__ bool chunk_of(const BMat &M, int64_t g, int64_t &dom, int64_t &ch) {
    if (g >= M.tchunks) return false;
    dom_of_chunk(M.pa, g, dom, ch);
    return true;
}

__global__ __launch_bounds__(256) void k_apply_p1_b(const BMat *__restrict__ mats, const int *__restrict__ list,
                                                    int sweep) {
    const BMat &M = mats[list[blockIdx.y]];
    int64_t dom, ch;
    if (!chunk_of(M, blockIdx.x, dom, ch)) return;
    if (sweep > 0 && M.status[1]) return;
    if (M.prec) apply_p1_body<TileF32>(M.V32, M.pa.m, M.pa, M.F, M.pa.m, 1, M.Pc, dom, ch);
    else apply_p1_body<TileF64>(M.V, M.pa.m, M.pa, M.F, M.pa.m, 1, M.Pc, dom, ch);
}

__global__ __launch_bounds__(256) void k_apply_p2_b(const BMat *__restrict__ mats, const int *__restrict__ list,
                                                    int trans, int sweep) {
    const BMat &M = mats[list[blockIdx.y]];
    if ((int64_t)blockIdx.x >= M.pa.P) return;
    if (sweep > 0 && M.status[1]) return;
    apply_p2_body(M.V, M.V32, M.pa.m, M.Tc, M.pa, M.F, M.pa.m, 1, trans, M.Pc, M.Zc, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_apply_p3_b(const BMat *__restrict__ mats, const int *__restrict__ list,
                                                    int sweep) {
    const BMat &M = mats[list[blockIdx.y]];
    int64_t dom, ch;
    if (!chunk_of(M, blockIdx.x, dom, ch)) return;
    if (sweep > 0 && M.status[1]) return;
    if (M.prec) apply_p3_body<TileF32>(M.V32, M.pa.m, M.pa, M.F, M.pa.m, 1, M.Zc, dom, ch);
    else apply_p3_body<TileF64>(M.V, M.pa.m, M.pa, M.F, M.pa.m, 1, M.Zc, dom, ch);
}

hipError_t launch_apply3_b(const BMat *mats, const int *list, int cnt, int64_t max_chunks, int64_t max_p,
                           int trans, int sweep, hipStream_t st) {
    if (cnt <= 0 || max_chunks <= 0) return hipSuccess;
    const size_t sh = vtb_lds_bytes<TileF64>(1);   // k = 1
    hipError_t e = hipFuncSetAttribute((const void *)k_apply_p1_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sh);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_apply_p2_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sizeof(ChainSmem));
    if (e != hipSuccess) return e;
    {
        ProfScope ps(trans ? "batch_apply3_p1_qt" : "batch_apply3_p1_q", st);
        hipLaunchKernelGGL(k_apply_p1_b, dim3((unsigned)max_chunks, (unsigned)cnt), dim3(256), sh, st, mats, list,
                           sweep);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope ps(trans ? "batch_apply3_p2_qt" : "batch_apply3_p2_q", st);
        hipLaunchKernelGGL(k_apply_p2_b, dim3((unsigned)max_p, (unsigned)cnt), dim3(256), sizeof(ChainSmem), st,
                           mats, list, trans, sweep);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    ProfScope ps(trans ? "batch_apply3_p3_qt" : "batch_apply3_p3_q", st);
    hipLaunchKernelGGL(k_apply_p3_b, dim3((unsigned)max_chunks, (unsigned)cnt), dim3(256), 0, st, mats, list,
                       sweep);
    return hipGetLastError();
}

template <typename Tile>
static hipError_t launch_apply3(const typename Tile::T *V, const double *V64, const float *V32, int64_t ldv,
                                const double *Tc, const PanelArgs &pa, double *B, int64_t ldb, int64_t k,
                                int trans, double *Pc, double *Zc, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const size_t sh = vtb_lds_bytes<Tile>(k);
    hipError_t e = hipFuncSetAttribute((const void *)k_apply_p1<Tile>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_apply_p2, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sizeof(ChainSmem));
    if (e != hipSuccess) return e;
    const dim3 chunks((unsigned)max_domain_chunks(pa), (unsigned)pa.P);
    {
        ProfScope ps(trans ? "apply3_p1_qt" : "apply3_p1_q", st);
        hipLaunchKernelGGL(k_apply_p1<Tile>, chunks, dim3(256), sh, st, V, ldv, pa, B, ldb, k, Pc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope ps(trans ? "apply3_p2_qt" : "apply3_p2_q", st);
        hipLaunchKernelGGL(k_apply_p2, dim3((unsigned)pa.P), dim3(256), sizeof(ChainSmem), st, V64, V32, ldv,
                           Tc, pa, B, ldb, k, trans, Pc, Zc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    ProfScope ps(trans ? "apply3_p3_qt" : "apply3_p3_q", st);
    hipLaunchKernelGGL(k_apply_p3<Tile>, chunks, dim3(256), 0, st, V, ldv, pa, B, ldb, k, Zc);
    return hipGetLastError();
}

hipError_t launch_leaf_apply3(const double *V, int64_t ldv, const double *Tc, const PanelArgs &pa, double *B,
                              int64_t ldb, int64_t k, int trans, double *Pc, double *Zc, hipStream_t st) {
    return launch_apply3<TileF64>(V, V, nullptr, ldv, Tc, pa, B, ldb, k, trans, Pc, Zc, st);
}

hipError_t launch_leaf_apply3_32(const float *V, int64_t ldv, const double *Tc, const PanelArgs &pa,
                                 double *B, int64_t ldb, int64_t k, int trans, double *Pc, double *Zc,
                                 hipStream_t st) {
    return launch_apply3<TileF32>(V, nullptr, V, ldv, Tc, pa, B, ldb, k, trans, Pc, Zc, st);
}

}  // namespace tsqr
