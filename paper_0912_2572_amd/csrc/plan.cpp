// plan.cpp -- domain partition, tree schedule, panels and workspace layout.
//
// Partition (Sec. 2.3, "the TS matrix is split in P block-rows, called
// domains"): P = ceil(m / mb) contiguous domains; a last domain with fewer
// than n rows is merged into the one before it so that every domain's QR has
// n reflectors.  Trees (Sec. 2.3): binary (adjacent pairs per level), k-ary
// (groups of k consecutive live nodes reduced left to right) and flat
// (R <- comb(R, R_i) for i = 1..P-1), and the hierarchical tree (each XCD's
// domains first, then across the XCDs; plan.h); results stay in the lower
// index.
// Matrices wider than 64 columns are factored in 64-column panels, each a
// TSQR of the rows that remain below the previous panels, with the panel's
// Q^T applied to the columns to its right in between: the factor-panel /
// update-trailing-matrix structure of CAQR (Sec. 2.3), which is also how the
// paper's ScaLAPACK domain kernel blocks its columns (block size 64, Sec. 5.2).
#include "plan.h"

#include <algorithm>

namespace tsqr {

static size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

std::vector<TreeLevel> tree_levels(int64_t P, int tree) {
    std::vector<TreeLevel> lv;
    if (P <= 1) return lv;
    if (tree == TSQR_TREE_FLAT) {
        lv.push_back(TreeLevel{1, P, 1, P - 1, 1});
        return lv;
    }
    if (tree == TSQR_TREE_XCD) {
        // inside each XCD: members x, x + G, x + 2G, ... paired as a binary
        // tree (chain g: left = (g / G) 2s + g % G, right = left + s)
        for (int64_t s = kXcds; s < P; s *= 2) {
            TreeLevel L;
            L.stride = s;
            L.span = 2 * s;
            L.width = kXcds;
            L.chains = ((P - s + L.span - 1) / L.span) * kXcds;
            L.max_rights = 1;
            lv.push_back(L);
        }
        // across the XCDs: the roots 0 .. min(P, G) - 1
        const int64_t roots = P < kXcds ? P : kXcds;
        for (int64_t s = 1; s < roots; s *= 2) {
            TreeLevel L;
            L.stride = s;
            L.span = 2 * s;
            L.width = 1;
            L.chains = (roots - s + L.span - 1) / L.span;
            L.max_rights = 1;
            lv.push_back(L);
        }
        return lv;
    }
    int64_t k = (tree == TSQR_TREE_QUAD) ? 4 : 2;
    for (int64_t stride = 1; stride < P; stride *= k) {
        TreeLevel L;
        L.stride = stride;
        L.span = stride * k;
        L.chains = (P - stride + L.span - 1) / L.span;
        L.max_rights = k - 1;
        lv.push_back(L);
    }
    return lv;
}

std::vector<std::pair<int64_t, int64_t>> tree_schedule(int64_t P, int tree) {
    std::vector<std::pair<int64_t, int64_t>> s;
    for (const TreeLevel &L : tree_levels(P, tree))
        for (int64_t g = 0; g < L.chains; ++g) {
            const int64_t left = (g / L.width) * L.span + g % L.width;
            for (int64_t q = 1; q * L.stride < L.span && left + q * L.stride < P; ++q)
                s.emplace_back(left, left + q * L.stride);
        }
    return s;
}

static int64_t default_row_block(int64_t m, int64_t n) {
    // Enough domains to give every one of the 256 compute units two
    // workgroups, rounded up to whole chunks, within [max(n, chunk), 8192].
    int64_t c = chunk_rows_for((int)std::min<int64_t>(n, kMaxPanel));
    int64_t want = (m + 511) / 512;
    int64_t mb = (want + c - 1) / c * c;
    mb = std::min<int64_t>(mb, std::max<int64_t>(8192, c));
    mb = std::max<int64_t>(mb, std::max<int64_t>(n, c));
    return mb;
}

// Load-balanced partition (Sec. 3: rows per domain in proportion to the
// processing power behind it; the compute units of one GPU are equal, so
// the shares are equal): the panel's C = ceil(m / chunk) chunks are split
// into P domains of C / P chunks, the first C mod P of them one chunk longer;
// the last domain ends at row m.  P is cut to C, and further while the last
// domain would hold fewer than n rows.
static void balance_panel(Panel &pa, int64_t want) {
    const int64_t C = (pa.m + pa.chunk - 1) / pa.chunk;
    int64_t P = want < C ? want : C;
    int64_t q = 0, e = 0;
    for (;; --P) {
        q = C / P;
        e = C % P;
        const int64_t last = pa.m - pa.chunk * ((P - 1) * q + e);
        if (P == 1 || last >= pa.n) break;
    }
    pa.P = P;
    pa.mb = q * pa.chunk;
    pa.extra = e;
    pa.cpd = q;
}

// Weighted partition (Sec. 3: rows per domain in proportion to the
// processing power behind it): the panel's C = ceil(m / chunk) chunks are
// apportioned to the integer powers w by largest remainders -- domain d gets
// floor(C w_d / W) chunks, and the chunks left over go one each to the
// domains with the largest C w_d mod W, ties to the lower index.  Returns
// false when a domain would get no chunk or fewer than n rows.
static bool weigh_panel(Panel &pa, const int64_t *w, int64_t P) {
    const int64_t C = (pa.m + pa.chunk - 1) / pa.chunk;
    int64_t W = 0;
    for (int64_t d = 0; d < P; ++d) {
        if (w[d] < 1 || w[d] > kMaxWeight) return false;   // C w_d and W stay in 64 bits
        W += w[d];
    }
    std::vector<int64_t> k(P), rem(P);
    int64_t given = 0;
    for (int64_t d = 0; d < P; ++d) {
        k[d] = C * w[d] / W;
        rem[d] = C * w[d] % W;
        given += k[d];
    }
    // the leftover chunks, largest remainder first (a stable order keeps
    // equal remainders in index order)
    std::vector<int64_t> order(P);
    for (int64_t d = 0; d < P; ++d) order[d] = d;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return rem[a] > rem[b]; });
    for (int64_t i = 0; i < C - given; ++i) k[order[i]] += 1;
    pa.wchunk0.assign(P + 1, 0);
    for (int64_t d = 0; d < P; ++d) {
        if (k[d] < 1) return false;
        pa.wchunk0[d + 1] = pa.wchunk0[d] + k[d];
    }
    pa.P = P;
    pa.mb = k[0] * pa.chunk;
    pa.cpd = 0;
    for (int64_t d = 0; d < P; ++d) pa.cpd = std::max(pa.cpd, k[d]);
    pa.extra = 0;
    for (int64_t d = 0; d < P; ++d)
        if (pa.domain_rows(d) < pa.n) return false;
    return true;
}

// Leaf workgroups one compute unit holds at once: two for panels of up to 32
// columns (their leaf fits two in registers and LDS), one for wider ones.
static int64_t leaf_residency(int n) { return n <= 32 ? 2 : 1; }

int make_plan(int64_t m, int64_t n, const tsqr_opts *o, Plan *p) {
    tsqr_opts d;
    tsqr_default_opts(&d);
    if (!o) o = &d;
    if (n < 1) return -2;
    if (m < n || m > 2147483647LL) return -1;
    if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
    if (o->tree != TSQR_TREE_FLAT && o->tree != TSQR_TREE_BINARY && o->tree != TSQR_TREE_QUAD &&
        o->tree != TSQR_TREE_XCD)
        return -5;
    if (o->prec != TSQR_F64 && o->prec != TSQR_MIXED) return -5;
    if (o->prec == TSQR_MIXED && n > kMaxMixedN) return TSQR_ERR_UNSUPPORTED;
    if (o->row_block != 0 && o->row_block < n) return -5;
    if (o->domains < -1 || (o->domains != 0 && o->row_block != 0)) return -5;
    if (!(o->route_kappa >= 0.0)) return -5;
    if (o->domain_weights &&
        (o->num_weights < 1 || o->num_weights > kMaxWeight || o->row_block != 0 || o->domains != 0))
        return -5;
    if (o->lsq_max_rhs < 1 || o->refine_max_iter < 0) return -5;
    Plan P;
    P.m = m;
    P.n = n;
    P.opts = *o;
    P.mb = o->row_block ? o->row_block : default_row_block(m, n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    P.off_w = take(sizeof(double) * (size_t)m * n);
    if (o->prec == TSQR_MIXED) P.off_w32 = take(sizeof(float) * (size_t)m * n);
    P.off_r = take(sizeof(double) * (size_t)n * n);
    P.off_d = take(sizeof(double) * (size_t)n);
    int np = (int)((n + kMaxPanel - 1) / kMaxPanel);
    for (int q = 0; q < np; ++q) {
        Panel pa;
        pa.col_off = q * kMaxPanel;
        pa.row_off = pa.col_off;
        pa.n = (int)std::min<int64_t>(kMaxPanel, n - pa.col_off);
        pa.m = m - pa.row_off;
        pa.ns = slots_for(pa.n);
        pa.chunk = chunk_rows_for(pa.n);
        if (o->domain_weights) {
            if (!weigh_panel(pa, o->domain_weights, o->num_weights)) return -5;
        } else if (o->domains != 0) {
            balance_panel(pa, o->domains > 0 ? o->domains : kComputeUnits * leaf_residency(pa.n));
        } else {
            pa.mb = P.mb;
            if (pa.mb < pa.n) pa.mb = pa.n;
            pa.P = (pa.m + pa.mb - 1) / pa.mb;
            if (pa.P > 1 && pa.m - (pa.P - 1) * pa.mb < pa.n) pa.P -= 1;
            pa.cpd = (pa.mb + pa.chunk - 1) / pa.chunk;
        }
        pa.total_chunks = pa.domain_chunk0(pa.P - 1) + pa.domain_chunks(pa.P - 1);
        pa.maxch = std::max(pa.domain_chunks(pa.P - 1), pa.P > 1 ? pa.domain_chunks(0) : (int64_t)0);
        for (int64_t d = 1; d + 1 < pa.P && !pa.wchunk0.empty(); ++d)
            pa.maxch = std::max(pa.maxch, pa.domain_chunks(d));
        pa.tree = o->tree;
        size_t nn = (size_t)pa.n * pa.n * sizeof(double);
        pa.off_tc = take(nn * (size_t)pa.total_chunks);
        pa.off_rdom = take(nn * (size_t)pa.P);
        pa.off_tnode = take(nn * (size_t)pa.P);
        pa.off_s = take(nn * (size_t)pa.P);
        if (o->keep_q) pa.off_pz = take(2 * sizeof(double) * (size_t)pa.n * 16 * (size_t)pa.total_chunks);
        if (!pa.wchunk0.empty()) pa.off_wtab = take(sizeof(int64_t) * pa.wchunk0.size());
        P.panels.push_back(pa);
    }
    P.off_lsq = take(sizeof(double) * (size_t)m * o->lsq_max_rhs);
    if (o->prec == TSQR_MIXED) {
        P.off_lsq2 = take(sizeof(double) * (size_t)m * o->lsq_max_rhs);
        // x (n x k), per-block A^T r partials (blocks x n x k), per-block
        // squared residual norms (blocks x 2k), last relative corrections
        // and ||A^T r|| (2k), backward-error bounds (k), flags
        const size_t k = (size_t)o->lsq_max_rhs;
        P.off_ref = take(sizeof(double) * (n * k + (size_t)kRefineBlocks * (n + 2) * k + 3 * k) + 64);
    }
    // small scratch: per-block partial sums (4096 blocks x rhs), a few
    // n x rhs vectors, info words and counters
    P.off_cond = take(sizeof(double));
    P.small_bytes = sizeof(double) * (size_t)(4096 + 8 * n) * o->lsq_max_rhs + 4096;
    P.off_small = take(P.small_bytes);
    P.total = off;
    *p = P;
    return 0;
}

}  // namespace tsqr
