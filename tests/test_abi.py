"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/tsqr.h declares, plans like the oracle partitions,
and rejects invalid arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsqr.h")
LIB = os.path.join(ROOT, "paper_0912_2572_amd", "libtsqr.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"TSQR_API\s+[\w\s\*]+?\b(tsqr_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def tl():
    if not os.path.exists(LIB):
        import paper_0912_2572_amd.build as b
        b.build()
    import paper_0912_2572_amd as t
    return t


def test_header_declares_the_four_calls():
    syms = declared_symbols()
    for s in ("tsqr_factor", "tsqr_apply_qt", "tsqr_form_q", "tsqr_lsq_solve"):
        assert s in syms


def test_library_exports_every_declared_symbol(tl):
    L = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_plan_matches_oracle_partition(tl):
    for m, n, mb in [(4096, 16, 1024), (1 << 20, 64, 4096), (1010, 16, 500), (5003, 13, 700),
                     (777, 1, 100), (64, 64, 64)]:
        P, chunk, npan = tl.plan_info(m, n, tl.opts(row_block=mb))
        assert P == len(oracle.partition(m, n, mb))
        assert npan == 1
        assert chunk >= n


def test_partition_query_matches_oracle(tl):
    for m, n, mb in [(4096, 16, 1024), (1 << 20, 64, 4096), (1010, 16, 500), (5003, 13, 700),
                     (777, 1, 100), (64, 64, 64)]:
        assert tl.partition(m, n, tl.opts(row_block=mb)) == oracle.partition(m, n, mb)


# (m, n, requested domains): several chunks per domain, a remainder spread
# over the first domains, more domains than chunks, a last domain that would
# be shorter than n, and the widths of all three leaf chunk sizes
BALANCED = [(1_200_000, 64, 256), (300_000, 64, 256), (5003, 13, 7), (100_000, 20, 100),
            (70_000, 32, 512), (2000, 64, 16), (1034, 24, 4), (1 << 20, 64, 256), (999, 64, 1)]


@pytest.mark.parametrize("m,n,want", BALANCED)
def test_balanced_partition_is_the_oracle_equal_power_partition(tl, m, n, want):
    """opts.domains: P domains of whole leaf chunks apportioned to equal
    powers -- the oracle's load-balanced partition (Sec. 3) with one weight
    per domain -- with P cut to the chunk count and while the last domain
    would be shorter than n."""
    P, chunk, _ = tl.plan_info(m, n, tl.opts(domains=want))
    got = tl.partition(m, n, tl.opts(domains=want))
    assert len(got) == P
    assert got == oracle.partition_weighted(m, n, P, chunk)
    C = -(-m // chunk)
    expect = min(want, C)
    while expect > 1:
        try:
            oracle.partition_weighted(m, n, expect, chunk)
            break
        except ValueError:
            expect -= 1
    assert P == expect
    sizes = [nr for _, nr in got[:-1]]
    assert not sizes or max(sizes) - min(sizes) <= chunk


@pytest.mark.parametrize("m,n,weights", [
    (100_000, 64, [1, 2, 3, 4]),
    (1_200_000, 64, [2, 1] * 128),              # half the power on every other domain
    (300_001, 20, [5, 5, 1, 1, 1, 3, 2] * 10),  # ties among the remainders
    (5003, 13, [1, 1, 1]),
    (70_000, 130, [4, 3, 2, 1]),                # three panels, each weighted over its rows
])
def test_weighted_partition_is_the_oracle_apportionment(tl, m, n, weights):
    o = tl.opts(weights=weights)
    P, chunk, _ = tl.plan_info(m, n, o)
    assert P == len(weights)
    assert tl.partition(m, n, o) == oracle.partition_weighted(m, n, P, chunk, weights)
    assert tl.workspace_bytes(m, n, o) > 8 * m * n


def test_weighted_partition_rejected_cases(tl):
    L = tl.lib()
    for bad in (tl.opts(weights=[1, 0, 2]),                    # a domain of no power
                tl.opts(weights=[1, 2], row_block=4096),       # with row_block
                tl.opts(weights=[1, 2], domains=8),            # with domains
                tl.opts(weights=[1000, 1]),                    # a domain without a chunk
                tl.opts(weights=[1, 1 << 40])):                # a weight past 2^31
        assert L.tsqr_partition(100_000, 16, ctypes.byref(bad), None, None, 0) == -5
    o = tl.opts(weights=[1, 1])
    o.num_weights = 0
    assert L.tsqr_partition(100_000, 16, ctypes.byref(o), None, None, 0) == -5
    d = ctypes.c_void_p(256)
    o = tl.opts(weights=[1, 1])
    assert L.tsqr_factor_solve_noalloc(1000, 8, d, 1000, ctypes.byref(o), 1, d, 1000, d, 8, None, None,
                                       None, 1000, None, 8, None) == tl.ERR_UNSUPPORTED


def test_balanced_partition_defaults_to_one_domain_per_resident_leaf(tl):
    for n, per_cu in [(8, 2), (16, 2), (32, 2), (33, 1), (64, 1), (128, 1)]:
        P, chunk, _ = tl.plan_info(1 << 22, n, tl.opts(domains=-1))
        assert P == 256 * per_cu
        assert tl.partition(1 << 22, n, tl.opts(domains=-1)) == oracle.partition_weighted(1 << 22, n, P, chunk)
    # a wide matrix balances each 64-column panel over its own rows
    assert tl.plan_info(300_000, 200, tl.opts(domains=256))[2] == 4
    assert tl.workspace_bytes(300_000, 200, tl.opts(domains=256)) > 8 * 300_000 * 200


def test_wide_problems_are_split_in_64_column_panels(tl):
    for n, want in [(64, 1), (65, 2), (128, 2), (200, 4), (256, 4)]:
        assert tl.plan_info(100000, n, tl.opts(row_block=4096))[2] == want


@pytest.mark.parametrize("tree", [0, 2, 4])
@pytest.mark.parametrize("P", [1, 2, 5, 8, 17, 256])
def test_tree_schedule_matches_oracle(tl, tree, P):
    assert tl.tree_schedule(P, tree) == oracle.schedule(P, tree)


@pytest.mark.parametrize("P", [1, 2, 5, 8, 9, 17, 64, 255, 256, 1024])
def test_xcd_tree_schedule(tl, P):
    """The hierarchical tree (TSQR_TREE_XCD): the same combines as the
    oracle's grid-tuned tree with domain d in cluster d mod 8, executed in
    an order the dependencies allow (a right is never used again, a left is
    used only after everything combined into it below), and XCD count - 1
    combines across an XCD boundary."""
    s = tl.tree_schedule(P, tl.TREE_XCD)
    want = oracle.hierarchical_schedule([d % 8 for d in range(P)])
    assert sorted(s) == sorted(want)
    done = set()
    for l, r in s:
        assert l < r and l not in done and r not in done
        done.add(r)
    assert sum(1 for l, r in s if l % 8 != r % 8) == min(P, 8) - 1
    assert len(tl.tree_schedule(P, tl.TREE_BINARY)) == len(s) == P - 1


def test_workspace_bytes(tl):
    o = tl.opts(row_block=4096)
    w = tl.workspace_bytes(1 << 20, 64, o)
    # the reflectors (m x n) plus, per 256-row chunk, its n x n T and the
    # few-column apply's two n x 16 blocks
    m, n, chunks = 1 << 20, 64, (1 << 20) // 256
    assert w >= 8 * m * n + 8 * chunks * (n * n + 2 * n * 16)
    assert w < 8 * m * n * 1.6
    assert tl.workspace_bytes(10, 20, o) == 0          # m < n
    assert tl.workspace_bytes(2000, 1100, o) == 0      # n above scope
    assert tl.workspace_bytes(2000, 1024, o) > 8 * 2000 * 1024
    assert tl.workspace_bytes(2000, 300, tl.opts(row_block=4096, prec=tl.MIXED)) == 0   # mixed: n <= 256


def test_invalid_arguments_rejected_on_host(tl):
    L = tl.lib()
    o = tl.opts(row_block=64)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    assert L.tsqr_factor(10, 20, dummy, 10, ctypes.byref(o), dummy, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.tsqr_factor(100, 0, dummy, 100, ctypes.byref(o), dummy, 1 << 20, None, ctypes.byref(h)) == -2
    assert L.tsqr_factor(100, 4, None, 100, ctypes.byref(tl.opts(row_block=64)), dummy, 1 << 30, None,
                         ctypes.byref(h)) == -3
    assert L.tsqr_factor(100, 4, dummy, 99, ctypes.byref(o), dummy, 1 << 30, None, ctypes.byref(h)) == -4
    bad = tl.opts(row_block=3)
    assert L.tsqr_factor(100, 4, dummy, 100, ctypes.byref(bad), dummy, 1 << 30, None, ctypes.byref(h)) == -5
    bad = tl.opts(tree=3)
    assert L.tsqr_factor(100, 4, dummy, 100, ctypes.byref(bad), dummy, 1 << 30, None, ctypes.byref(h)) == -5
    for bad in (tl.opts(domains=-2), tl.opts(domains=4, row_block=64), tl.opts(route_kappa=-1.0),
                tl.opts(route_kappa=float("nan"))):
        assert L.tsqr_factor(100, 4, dummy, 100, ctypes.byref(bad), dummy, 1 << 30, None, ctypes.byref(h)) == -5
        assert L.tsqr_partition(100, 4, ctypes.byref(bad), None, None, 0) == -5
    assert L.tsqr_factor(100, 4, dummy, 100, ctypes.byref(o), None, 1 << 30, None,
                         ctypes.byref(h)) == tl.ERR_WORKSPACE
    assert L.tsqr_factor(100, 4, dummy, 100, ctypes.byref(o), dummy, 16, None,
                         ctypes.byref(h)) == tl.ERR_WORKSPACE
    assert L.tsqr_factor(2000, 1100, dummy, 2000, ctypes.byref(o), dummy, 1 << 30, None,
                         ctypes.byref(h)) == tl.ERR_UNSUPPORTED
    mixed = tl.opts(row_block=4096, prec=tl.MIXED)
    assert L.tsqr_factor(2000, 300, dummy, 2000, ctypes.byref(mixed), dummy, 1 << 30, None,
                         ctypes.byref(h)) == tl.ERR_UNSUPPORTED
    assert not h.value
    assert L.tsqr_strerror(-900).decode().startswith("workspace")


def test_batch_workspace_and_item_checks(tl):
    L = tl.lib()
    shapes = [(5000, 8), (20000, 64), (1000, 16)]
    w_default = tl.batch_workspace_bytes(shapes, [0, 1, 0],
                                         tune=[{"n_max": 64, "prec": 0, "row_block": 4096, "tree": 2},
                                               {"n_max": 64, "prec": 1, "row_block": 4096, "tree": 2}])
    w_space = tl.batch_workspace_bytes(shapes, [0, 1, 0])
    # reflectors: FP64 for matrices 0 and 2, FP32 for the mixed one
    assert w_default >= 8 * (5000 * 8 + 1000 * 16) + 4 * 20000 * 64
    assert w_space >= w_default
    # out of scope: n > 64 (batched matrices are single-panel), m < n
    assert tl.batch_workspace_bytes([(5000, 65)], [0]) == 0
    assert L.tsqr_batch_bad_item() == 0
    assert tl.batch_workspace_bytes([(100, 8), (10, 20)], [0, 0]) == 0
    assert L.tsqr_batch_bad_item() == 1
    assert tl.batch_workspace_bytes([(100, 8)], [2]) == 0   # unknown precision


def test_batch_create_rejects_on_host(tl):
    L = tl.lib()
    items = (tl.BatchItem * 1)()
    items[0].m, items[0].n, items[0].prec, items[0].lda = 1000, 8, 0, 1000
    h = ctypes.c_void_p()
    # NULL device pointers in the item: rejected before any device work
    assert L.tsqr_batch_create(1, items, None, 0, 2, 1e-14, ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(h)) == -2
    assert L.tsqr_batch_create(0, items, None, 0, 2, 1e-14, ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(h)) == -1
    assert L.tsqr_batch_create(1, items, None, 0, -1, 1e-14, ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(h)) == -5
    assert not h.value
    assert L.tsqr_autotune(1, items, 0, None, 0, None, None, 0) == -3


def test_tslu_arguments_checked_on_host(tl):
    L = tl.lib()
    o = tl.opts(row_block=1000)
    d = ctypes.c_void_p(256)
    w = tl.lib().tsqr_tslu_workspace_bytes(10000, 16, ctypes.byref(o))
    assert w >= 10 * 16 * 4
    assert L.tsqr_tslu_workspace_bytes(10000, 65, ctypes.byref(o)) == 0
    args = lambda m, b, lda, ldl, ldu: (m, b, d, lda, ctypes.byref(o), d, 1 << 30, d, ldl, d, ldu, d, None, None)
    assert L.tsqr_tslu(*args(10000, 65, 10000, 10000, 65)) == tl.ERR_UNSUPPORTED
    assert L.tsqr_tslu(*args(10000, 0, 10000, 10000, 1)) == -2
    assert L.tsqr_tslu(*args(10, 16, 10, 10, 16)) == -1
    assert L.tsqr_tslu(*args(10000, 16, 9999, 10000, 16)) == -4
    assert L.tsqr_tslu(*args(10000, 16, 10000, 9999, 16)) == -6
    assert L.tsqr_tslu(*args(10000, 16, 10000, 10000, 15)) == -7
    small = (10000, 16, d, 10000, ctypes.byref(o), d, 16, d, 10000, d, 16, d, None, None)
    assert L.tsqr_tslu(*small) == tl.ERR_WORKSPACE


def test_calu_arguments_checked_on_host(tl):
    L = tl.lib()
    o = tl.opts(row_block=512)
    d = ctypes.c_void_p(256)
    w = L.tsqr_calu_workspace_bytes(3000, 200, ctypes.byref(o))
    assert w >= 3000 * 64 * 8
    assert L.tsqr_calu_workspace_bytes(100, 200, ctypes.byref(o)) == 0
    assert L.tsqr_calu_workspace_bytes(100, 0, ctypes.byref(o)) == 0
    args = lambda m, n, A, lda, ipiv, info, wb: (m, n, A, lda, ctypes.byref(o), d, wb, ipiv, info, None)
    assert L.tsqr_calu(*args(100, 200, d, 100, d, d, w)) == -1
    assert L.tsqr_calu(*args(3000, 0, d, 3000, d, d, w)) == -2
    assert L.tsqr_calu(*args(3000, 200, None, 3000, d, d, w)) == -3
    assert L.tsqr_calu(*args(3000, 200, d, 2999, d, d, w)) == -4
    assert L.tsqr_calu(*args(3000, 200, d, 3000, None, d, w)) == -8
    assert L.tsqr_calu(*args(3000, 200, d, 3000, d, None, w)) == -9
    assert L.tsqr_calu(*args(3000, 200, d, 3000, d, d, 16)) == tl.ERR_WORKSPACE
    wts = np.array([1, 2, 3], dtype=np.int64)
    ow = tl.opts(weights=wts)
    assert L.tsqr_calu_workspace_bytes(3000, 200, ctypes.byref(ow)) == 0
    assert L.tsqr_calu(3000, 200, d, 3000, ctypes.byref(ow), d, w, d, d, None) == tl.ERR_UNSUPPORTED


def test_cholesky_arguments_checked_on_host(tl):
    L = tl.lib()
    d = ctypes.c_void_p(256)
    assert L.tsqr_cholesky(-1, d, 1, d, None) == -1
    assert L.tsqr_cholesky(10, None, 10, d, None) == -2
    assert L.tsqr_cholesky(10, d, 9, d, None) == -3
    assert L.tsqr_cholesky(0, None, 0, d, None) == -3
    assert L.tsqr_cholesky(10, d, 10, None, None) == -4
    assert L.tsqr_cholesky(1 << 31, d, 1 << 31, d, None) == tl.ERR_UNSUPPORTED


def test_routing_calls_check_their_handle(tl):
    L = tl.lib()
    prec, kap = ctypes.c_int32(), ctypes.c_double()
    assert L.tsqr_route_info(None, ctypes.byref(prec), ctypes.byref(kap)) == -1
    assert L.tsqr_cond_estimate(None, ctypes.c_void_p(256), None) == -1
    o = tl.ServerOpts()
    L.tsqr_server_default_opts(ctypes.byref(o))
    assert o.route_kappa == 1e4
    o.route_kappa = -1.0
    h = ctypes.c_void_p()
    assert L.tsqr_server_create(ctypes.byref(o), ctypes.byref(h)) == -1 and not h.value


def test_server_options_checked_on_host(tl):
    L = tl.lib()
    o = tl.ServerOpts()
    L.tsqr_server_default_opts(ctypes.byref(o))
    assert o.streams >= 1 and o.max_inflight >= 1 and o.cache == 1
    h = ctypes.c_void_p()
    o.streams = 0
    assert L.tsqr_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    L.tsqr_server_default_opts(ctypes.byref(o))
    o.hbm_budget = 1000
    assert L.tsqr_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    L.tsqr_server_default_opts(ctypes.byref(o))
    o.prec = 5
    assert L.tsqr_server_create(ctypes.byref(o), ctypes.byref(h)) == -1
    assert not h.value
    assert L.tsqr_server_submit(None, None) == -1
