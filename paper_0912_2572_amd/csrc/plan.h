// plan.h -- host-side plan of a TSQR factorization: domain partition, leaf
// chunking, tree schedule, 64-column panels and the workspace layout.
// Pure C++ (no device code), so the plan is testable on a machine without a
// GPU through tsqr_plan_info / tsqr_workspace_bytes.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/tsqr.h"
#include "common.h"

namespace tsqr {

constexpr int kMaxPanel = 64;     // columns handled by one leaf/tree kernel
constexpr int kMaxN = 1024;       // documented scope (FP64)
constexpr int kMaxMixedN = 256;   // mixed precision (the refinement's one-wave solves)
constexpr int kThreads = 256;     // threads per workgroup of the leaf kernel
constexpr size_t kAlign = 256;
constexpr int kRefineBlocks = 1024;   // workgroups of the refinement's residual pass
constexpr int64_t kComputeUnits = 256;  // compute units of one gfx950 GPU (MI355X)
constexpr int64_t kMaxWeight = (int64_t)1 << 31;  // largest domain weight, and weight count

// Column slots per thread of the leaf kernel for a panel of width w: 16
// column groups x ns slots must cover w (ns = 1, 2 or 4).  Rows per chunk
// are the device tile's (common.h: 512 for ns = 1 and 4, 256 for ns = 2).
inline int slots_for(int w) {
    int need = (w + 15) / 16;
    int ns = 1;
    while (ns < need) ns <<= 1;
    return ns;
}
inline int chunk_rows_for(int w) { return chunk_rows(slots_for(w)); }

// One TSQR over rows [row_off, row_off + m) and columns [col_off, col_off+n)
// of the working matrix (n <= 64).
struct Panel {
    int64_t m = 0, row_off = 0;
    int n = 0, col_off = 0;
    int64_t mb = 0, P = 0;          // domains of mb rows (the last one ragged)
    int64_t extra = 0;              // load-balanced partition: domains 0 .. extra-1
                                    // hold one chunk more than mb (mb whole chunks)
    int ns = 0;                     // slots per thread (1, 2, 4, 8)
    int64_t chunk = 0;              // rows per chunk of the leaf kernel
    int64_t cpd = 0;                // chunks in a full domain
    int64_t total_chunks = 0;
    int64_t maxch = 0;              // most chunks of any domain
    int tree = TSQR_TREE_BINARY;
    // workspace offsets (bytes from the workspace base)
    size_t off_tc = 0;              // total_chunks x n x n   (chunk T factors)
    size_t off_rdom = 0;            // P x n x n              (domain R / node U)
    size_t off_tnode = 0;           // P x n x n              (node T, by right child)
    size_t off_s = 0;               // P x n x n              (top-down blocks)
    size_t off_pz = 0;              // 2 x total_chunks x n x 16 (few-column apply: P_c, Z_c)
    // weighted partition (opts.domain_weights): first chunk of every domain,
    // P + 1 entries (the last = the panel's chunk count), on the host and,
    // copied there by the factorization, in the workspace
    std::vector<int64_t> wchunk0;
    size_t off_wtab = 0;

    int64_t domain_row0(int64_t i) const {
        if (!wchunk0.empty()) return wchunk0[i] * chunk;
        return i * mb + (i < extra ? i : extra) * chunk;
    }
    int64_t domain_rows(int64_t i) const {
        if (i == P - 1) return m - domain_row0(i);
        if (!wchunk0.empty()) return (wchunk0[i + 1] - wchunk0[i]) * chunk;
        return mb + (i < extra ? chunk : 0);
    }
    int64_t domain_chunk0(int64_t i) const {
        if (!wchunk0.empty()) return wchunk0[i];
        return i * cpd + (i < extra ? i : extra);
    }
    int64_t domain_chunks(int64_t i) const { return (domain_rows(i) + chunk - 1) / chunk; }
};

// Tree levels: one kernel launch per level, one workgroup per chain.  A chain
// is (left, right_1, ..., right_c): the rights are combined into left one
// after the other (binary: c = 1, k-ary: c = k - 1, flat: one chain of P - 1).
// Chain g of a level starts at left = (g / width) span + g % width.
struct TreeLevel {
    int64_t stride = 0;    // distance between consecutive rights of a chain
    int64_t span = 0;      // distance between consecutive groups of lefts
    int64_t chains = 0;
    int64_t max_rights = 0;
    int64_t width = 1;     // lefts per group (consecutive indices)
};

// The hierarchical tree (TSQR_TREE_XCD) groups domain d with the domains of
// its XCD: leaves are dispatched round-robin over the XCDs, so domain d runs
// on XCD d mod kXcds.  A binary tree reduces each XCD's domains first (their
// triangles stay in that XCD's L2), then a binary tree reduces the kXcds
// roots 0 .. kXcds - 1: kXcds - 1 combines cross an XCD boundary, the
// grid-tuned tree of the paper's Sec. 2.3 (Fig. 2) with an XCD as a cluster.
constexpr int64_t kXcds = 8;
std::vector<TreeLevel> tree_levels(int64_t P, int tree);
// The flat list of (left, right) combines in execution order, for tests.
std::vector<std::pair<int64_t, int64_t>> tree_schedule(int64_t P, int tree);

struct Plan {
    int64_t m = 0, n = 0;
    tsqr_opts opts{};
    int64_t mb = 0;
    std::vector<Panel> panels;
    size_t off_w = 0;       // m x n FP64 working matrix (reflectors, trailing updates)
    size_t off_w32 = 0;     // m x n FP32 copy of the reflectors (mixed only)
    size_t off_r = 0;       // n x n final R
    size_t off_d = 0;       // n signs
    size_t off_lsq = 0;     // m x lsq_max_rhs scratch (Q^T B)
    size_t off_lsq2 = 0;    // m x lsq_max_rhs scratch (refinement residual)
    size_t off_ref = 0;     // refinement scratch (mixed only): x, partial sums, flags
    size_t off_cond = 0;    // one double: the condition estimate of mixed-precision routing
    size_t off_small = 0;   // small scratch: partial sums, x corrections, info words
    size_t small_bytes = 0;
    size_t total = 0;
};

// Returns 0 and fills *p, or a negative argument code.
int make_plan(int64_t m, int64_t n, const tsqr_opts *o, Plan *p);

}  // namespace tsqr
