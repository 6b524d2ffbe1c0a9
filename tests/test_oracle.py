"""Pins for the FP64 CPU oracle (runs without a GPU).

Each test ties the oracle to something other than itself: LAPACK routines
with the same conventions (called through SciPy, never read), exact rational
arithmetic, closed forms, and invariants that Agullo et al. state for TSQR:
uniqueness of R with a positive diagonal (Sec. 2.2) and associativity /
commutativity of the R-combine (Sec. 2.3).  A dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.lapack as lapack

import oracle
import synth

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def signfix(R):
    d = np.where(np.diag(R) < 0, -1.0, 1.0)
    return d[:, None] * R


# ---------------------------------------------------------------- reflector

@pytest.mark.parametrize("alpha,n", [(0.7, 9), (-1.3, 5), (0.0, 6), (2.5, 1)])
def test_larfg_matches_lapack_and_annihilates(alpha, n):
    rng = np.random.default_rng(11 + n)
    x = rng.standard_normal(n)
    beta, v, tau = oracle.larfg(alpha, x)
    lb, lv, lt = lapack.dlarfg(n + 1, alpha, x.copy())
    assert abs(beta - lb) <= 8 * U * abs(lb)
    assert abs(tau - lt) <= 8 * U * max(abs(lt), 1e-300)
    assert rel(v, lv) <= 8 * U
    # H [alpha; x] = beta e_1 and H is orthogonal
    vv = np.concatenate([[1.0], v])
    H = np.eye(n + 1) - tau * np.outer(vv, vv)
    y = H @ np.concatenate([[alpha], x])
    assert abs(y[0] - beta) <= 16 * U * abs(beta)
    assert np.linalg.norm(y[1:]) <= 16 * U * abs(beta)
    assert np.linalg.norm(H.T @ H - np.eye(n + 1)) <= 32 * U


def test_larfg_negative_zero_alpha_uses_plus_sign():
    """sgn(0) = +1 for both signed zeros (reading of Sec. 2.2's reflector);
    LAPACK's Fortran SIGN treats -0.0 as negative, so this case is pinned by
    the reflector identity alone."""
    x = np.array([3.0, 4.0])
    beta, v, tau = oracle.larfg(-0.0, x)
    assert beta == -5.0 and tau == 1.0
    vv = np.concatenate([[1.0], v])
    y = (np.eye(3) - tau * np.outer(vv, vv)) @ np.array([0.0, 3.0, 4.0])
    assert np.allclose(y, [-5.0, 0.0, 0.0], atol=1e-15)


def test_larfg_zero_tail_is_identity():
    beta, v, tau = oracle.larfg(-3.0, np.zeros(4))
    assert tau == 0.0 and beta == -3.0 and np.all(v == 0.0)


# ------------------------------------------------------------- leaf (geqrt)

@pytest.mark.parametrize("r,n", [(50, 8), (17, 17), (64, 5), (9, 12)])
def test_geqrt_matches_lapack(r, n):
    rng = np.random.default_rng(r * 100 + n)
    A = rng.standard_normal((r, n))
    W, tau, T = oracle.geqrt(A)
    k = min(r, n)
    la, lt, info = lapack.dgeqrt(k, np.asfortranarray(A.copy()))
    assert info == 0
    assert rel(np.triu(W), np.triu(la)) <= 50 * U
    assert rel(np.tril(W, -1), np.tril(la, -1)) <= 200 * U
    assert rel(T[:k, :k], lt[:k, :k]) <= 200 * U


def test_geqrt_compact_wy_equals_product_of_reflectors():
    rng = np.random.default_rng(5)
    r, n = 40, 7
    A = rng.standard_normal((r, n))
    W, tau, T = oracle.geqrt(A)
    V = np.tril(W, -1)[:, :n] + np.eye(r, n)
    Q = np.eye(r)
    for j in range(n):
        v = V[:, j]
        Q = Q @ (np.eye(r) - tau[j] * np.outer(v, v))
    assert np.linalg.norm(Q - (np.eye(r) - V @ T @ V.T)) <= 64 * U
    assert rel(Q[:, :n] @ np.triu(W[:n]), A) <= 64 * U


# ---------------------------------------------------------- combine (tpqrt)

@pytest.mark.parametrize("n", [1, 4, 16])
def test_tpqrt_matches_lapack_and_dense_qr(n):
    rng = np.random.default_rng(300 + n)
    R1 = np.triu(rng.standard_normal((n, n)))
    R2 = np.triu(rng.standard_normal((n, n)))
    R, Uv, tau, T = oracle.tpqrt(R1, R2)
    la, lb, lt, info = lapack.dtpqrt(n, n, np.asfortranarray(R1.copy()), np.asfortranarray(R2.copy()))
    assert info == 0
    assert rel(np.triu(R), np.triu(la)) <= 50 * U
    assert rel(np.triu(Uv), np.triu(lb)) <= 200 * U
    assert rel(T, lt[:n, :n]) <= 200 * U
    # the structure-free computation: dense QR of the 2n x n stack
    Rd = np.linalg.qr(np.vstack([R1, R2]))[1]
    assert rel(signfix(np.triu(R)), signfix(Rd)) <= 50 * U
    # the reflectors really are [e_j; u_j]: applying them reproduces [R; 0]
    Y = np.vstack([np.eye(n), np.triu(Uv)])
    Q = np.eye(2 * n) - Y @ T @ Y.T
    assert rel(Q.T @ np.vstack([R1, R2]), np.vstack([np.triu(R), np.zeros((n, n))])) <= 64 * U


# ------------------------------------------------------- partition / trees

def test_partition_rule():
    assert oracle.partition(1000, 16, 300) == [(0, 300), (300, 300), (600, 300), (900, 100)]
    # a last domain shorter than n is merged into the one before it
    assert oracle.partition(1010, 16, 500) == [(0, 500), (500, 510)]
    assert oracle.partition(4096, 16, 1024) == [(0, 1024), (1024, 1024), (2048, 1024), (3072, 1024)]
    assert oracle.partition(16, 16, 16) == [(0, 16)]


def test_weighted_partition_worked_cases():
    # equal power: 10 granules over 3 domains, the one left over to domain 0
    assert oracle.partition_weighted(1000, 4, 3, 100) == [(0, 400), (400, 300), (700, 300)]
    # powers 1:2:1 of 10 granules: shares 2.5, 5, 2.5 -> 2, 5, 2 and the one
    # left over to the lower of the two tied remainders; the last granule
    # holds the 50 rows past 900
    assert oracle.partition_weighted(950, 4, 3, 100, [1, 2, 1]) == [(0, 300), (300, 500), (800, 150)]
    # half the cores of two of four machines (the paper's reservation case):
    # powers 2:1:2:1 of 12 granules -> 4, 2, 4, 2 exactly
    assert oracle.partition_weighted(1200, 8, 4, 100, [2, 1, 2, 1]) == [
        (0, 400), (400, 200), (600, 400), (1000, 200)]
    # granule 1: plain proportional rows
    assert oracle.partition_weighted(7, 1, 2, 1, [3, 4]) == [(0, 3), (3, 4)]
    # one domain holds everything
    assert oracle.partition_weighted(1234, 7, 1, 256) == [(0, 1234)]


def test_weighted_partition_rejects_empty_or_short_domains():
    with pytest.raises(ValueError):
        oracle.partition_weighted(1000, 4, 11, 100)          # 10 granules, 11 domains
    with pytest.raises(ValueError):
        oracle.partition_weighted(1000, 4, 2, 100, [1, 0])   # a domain of no power
    with pytest.raises(ValueError):
        oracle.partition_weighted(1010, 16, 2, 100, [10, 1])  # last domain: 10 rows < n
    with pytest.raises(ValueError):
        oracle.partition_weighted(1000, 4, 2, 100, [1, 2, 3])  # one weight per domain


@pytest.mark.parametrize("seed", range(6))
def test_weighted_partition_is_largest_remainder_apportionment(seed):
    """Brute-force check: contiguous cover of the rows, every domain's
    granule count is the floor or ceiling of its exact share C w_d / W, the
    counts sum to C, and the rounding-up goes to the largest remainders."""
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 40))
    g = int(rng.integers(1, 300))
    w = rng.integers(1, 20, size=P)
    C = int(rng.integers(int(w.sum()), 60 * int(w.sum())))   # every share >= 1 granule
    m = (C - 1) * g + int(rng.integers(1, g + 1))
    parts = oracle.partition_weighted(m, 1, P, g, w)
    assert parts[0][0] == 0 and parts[-1][0] + parts[-1][1] == m
    for (a, na), (b, _) in zip(parts, parts[1:]):
        assert a + na == b
    k = [nr // g for _, nr in parts[:-1]] + [C - sum(nr // g for _, nr in parts[:-1])]
    assert sum(k) == C
    W = int(w.sum())
    share = [Fraction(C * int(x), W) for x in w]
    up = [i for i in range(P) if k[i] > share[i]]
    for i in range(P):
        assert math.floor(share[i]) <= k[i] <= math.ceil(share[i])
    rem = [share[i] - math.floor(share[i]) for i in range(P)]
    down = [i for i in range(P) if k[i] == math.floor(share[i]) and rem[i] > 0]
    if up and down:
        assert min(rem[i] for i in up) >= max(rem[i] for i in down)


@pytest.mark.parametrize("m,n,P,g,w,tree", [
    (5003, 13, 7, 256, None, oracle.TREE_BINARY),
    (5003, 13, 5, 100, [1, 3, 2, 5, 1], oracle.TREE_BINARY),
    (9000, 20, 6, 64, [4, 4, 2, 2, 1, 1], oracle.TREE_FLAT),
    (3000, 25, 9, 128, None, oracle.TREE_QUAD),
])
def test_factor_over_a_weighted_partition(m, n, P, g, w, tree):
    """R, Q and Q^T B do not depend on the partition (Sec. 2.2 uniqueness of
    R with a positive diagonal): a weighted partition gives NumPy's
    sign-normalised QR, and its leaves are Householder QRs of exactly the
    apportioned rows."""
    rng = np.random.default_rng(m + P)
    A = rng.standard_normal((m, n))
    parts = oracle.partition_weighted(m, n, P, g, w)
    f = oracle.TSQR(A, parts=parts, tree=tree)
    assert f.P == P
    Qn, Rn = np.linalg.qr(A)
    d = np.where(np.diag(Rn) < 0, -1.0, 1.0)
    assert rel(f.R(), d[:, None] * Rn) <= 1e-13
    Q = f.form_q()
    for j in range(n):
        assert np.linalg.norm(Q[:, j] - Qn[:, j] * d[j]) <= 1e-12
    B = rng.standard_normal((m, 2))
    C = f.apply_qt(B)
    assert rel(C[:n], Q.T @ B) <= 1e-13
    # each leaf is the Householder QR of its own rows
    W, tau, _ = f.leaf()
    for i, (r0, nr) in enumerate(parts):
        la, ltau, _, _ = lapack.dgeqrf(np.asfortranarray(A[r0:r0 + nr].copy()))
        assert rel(np.triu(W[r0:r0 + n]), np.triu(la[:n])) <= 1e-13
        assert rel(tau[i], ltau) <= 1e-13


def test_factor_over_a_partition_rejects_gaps():
    A = np.ones((300, 2))
    with pytest.raises(ValueError):
        oracle.TSQR(A, parts=[(0, 100), (150, 150)])
    with pytest.raises(ValueError):
        oracle.TSQR(A, parts=[(0, 100), (100, 150)])      # stops short of m
    with pytest.raises(ValueError):
        oracle.TSQR(A, parts=[(0, 299), (299, 1)])        # a domain shorter than n


# ------------------------------------------------------------------- TSLU

def _lapack_pivot_rows(A):
    """The rows LAPACK's dgetrf picks as pivots, in order (its swaps replayed)."""
    lu, piv = scipy.linalg.lu_factor(A)
    perm = np.arange(A.shape[0])
    for i, p in enumerate(piv):
        perm[i], perm[p] = perm[p], perm[i]
    return perm[:A.shape[1]], lu


@pytest.mark.parametrize("m,b", [(1000, 8), (300, 1), (64, 64), (5000, 33)])
def test_tslu_one_stage_is_partial_pivoting(m, b):
    """One domain taken in one stage: the selection is GEPP's pivot sequence
    and U, L are dgetrf's (L's rows in A's order)."""
    A = np.random.default_rng(m + b).standard_normal((m, b))
    ipiv, L, U, info = oracle.tslu(A, [(0, m)], first=m, stage=1)
    pr, lu = _lapack_pivot_rows(A)
    assert info == 0
    assert ipiv.tolist() == pr.tolist()
    assert rel(U, np.triu(lu[:b])) <= 1e-13
    Ll = np.tril(lu, -1)[:, :b] + np.eye(m, b)
    perm = np.arange(m)
    _, piv = scipy.linalg.lu_factor(A)
    for i, p in enumerate(piv):
        perm[i], perm[p] = perm[p], perm[i]
    assert rel(L[perm], Ll) <= 1e-13


def test_tslu_every_node_selects_by_partial_pivoting():
    """Two domains in stages and a root: each stage's and the root's
    selection equal dgetrf's pivot rows on the stacked original rows."""
    rng = np.random.default_rng(3)
    m, b = 50, 3
    A = rng.standard_normal((m, b))
    parts = [(0, 20), (20, 30)]
    first, stage = 8, 5
    sel = []
    for r0, nr in parts:
        rows = list(range(r0, r0 + first))
        cur = [rows[i] for i in _lapack_pivot_rows(A[rows])[0]]
        pos = r0 + first
        while pos < r0 + nr:
            rows = cur + list(range(pos, min(pos + stage, r0 + nr)))
            cur = [rows[i] for i in _lapack_pivot_rows(A[rows])[0]]
            pos += stage
        sel.append(cur)
    rows = sel[0] + sel[1]
    root = [rows[i] for i in _lapack_pivot_rows(A[rows])[0]]
    ipiv, L, U, info = oracle.tslu(A, parts, first=first, stage=stage)
    assert ipiv.tolist() == root


@pytest.mark.parametrize("m,b,mb,first,stage,tree", [(20000, 16, 4096, 256, 240, oracle.TREE_BINARY),
                                                     (9001, 64, 1000, 256, 192, oracle.TREE_QUAD),
                                                     (3000, 5, 700, 100, 95, oracle.TREE_FLAT)])
def test_tslu_factorization_invariants(m, b, mb, first, stage, tree):
    """A = L U, L unit lower trapezoidal in the pivot order, |L| small
    (tournament pivoting keeps multipliers bounded in practice)."""
    A = np.random.default_rng(m).standard_normal((m, b))
    ipiv, L, U, info = oracle.tslu(A, oracle.partition(m, b, mb), first=first, stage=stage, tree=tree)
    assert info == 0 and len(set(ipiv.tolist())) == b
    assert np.linalg.norm(A - L @ U) <= 1e-14 * math.sqrt(m) * np.linalg.norm(A)
    assert np.all(np.tril(U, -1) == 0.0)
    L11 = L[ipiv]
    assert np.all(np.triu(L11, 1) == 0.0) and np.all(np.diag(L11) == 1.0)
    assert np.max(np.abs(L)) <= 20.0
    # the pivots of the root's stack came first: its U is the LU of A[ipiv]
    assert rel(L11 @ U, A[ipiv]) <= 1e-14


def test_tslu_exact_zero_column_info():
    A = np.random.default_rng(4).standard_normal((400, 6))
    A[:, 2] = 0.0
    ipiv, L, U, info = oracle.tslu(A, oracle.partition(400, 6, 100), first=50, stage=44)
    assert info == 3 and U[2, 2] == 0.0 and np.all(L[:, 2][np.setdiff1d(np.arange(400), ipiv)] == 0.0)


def test_tslu_integer_ties_go_to_the_lowest_row():
    # every |entry| of the first column equal: each search takes its first
    # active stack position, so the domain heads win
    A = np.ones((12, 2))
    A[:, 1] = np.arange(12) % 5
    ipiv, L, U, info = oracle.tslu(A, [(0, 6), (6, 6)], first=6, stage=1)
    assert ipiv[0] == 0


# ------------------------------------------------- condition of R (routing)

def _graded_r(n, decades, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3 * n + 5, n)) @ np.diag(10.0 ** np.linspace(0, -decades, n))
    return signfix(np.linalg.qr(A)[1])


@pytest.mark.parametrize("n,decades", [(1, 0), (2, 3), (7, 1), (16, 4), (64, 6), (129, 2), (256, 5)])
def test_cond1_is_numpys_one_norm_condition(n, decades):
    R = _graded_r(n, decades, n)
    assert oracle.cond1(R) == pytest.approx(np.linalg.cond(R, 1), rel=1e-9)


def test_cond1_special_cases():
    d = np.array([4.0, 0.5, 2.0, 8.0])
    assert oracle.cond1(np.diag(d)) == 8.0 / 0.5
    # a unit upper bidiagonal with -1 above the diagonal: R^{-1} is the
    # all-ones upper triangle, so ||R||_1 = 2 and ||R^{-1}||_1 = n
    n = 9
    R = np.eye(n) - np.diag(np.ones(n - 1), 1)
    assert oracle.cond1(R) == 2.0 * n
    R[3, 3] = 0.0
    assert oracle.cond1(R) == math.inf and oracle.cond1_est(R) == math.inf


@pytest.mark.parametrize("n,decades,seed", [(2, 3, 1), (5, 2, 2), (16, 4, 3), (64, 6, 4), (64, 0, 5),
                                             (100, 3, 6), (256, 5, 7)])
def test_cond1_estimate_is_a_lower_bound_at_least_lapacks(n, decades, seed):
    """The estimate never exceeds kappa_1 (it is ||R||_1 times ||R^{-1} x||_1
    for unit 1-norm vectors x) and is at least LAPACK's dtrcon estimate, the
    same method with the cycling test keeping the last value instead of the
    larger one; in practice it is within a small factor of kappa_1."""
    R = _graded_r(n, decades, seed)
    est, ex = oracle.cond1_est(R), oracle.cond1(R)
    rc, info = lapack.dtrcon(R, norm="1", uplo="U", diag="N")
    assert info == 0
    assert est <= ex * (1 + 1e-12)
    assert est >= (1.0 / rc) * (1 - 1e-12)
    assert est >= ex / 3


def test_cond1_estimate_exact_cases():
    # diagonal: the first sign vector is all +1, R^{-T} of it peaks at the
    # smallest |r_jj|, and that unit vector attains ||R^{-1}||_1
    d = np.array([3.0, 0.25, 7.0, 0.5, 2.0])
    assert oracle.cond1_est(np.diag(d)) == oracle.cond1(np.diag(d)) == 7.0 / 0.25
    assert oracle.cond1_est(np.array([[-2.5]])) == 1.0
    n = 12
    R = np.eye(n) - np.diag(np.ones(n - 1), 1)
    assert oracle.cond1_est(R) == oracle.cond1(R)


def _depth(sched, P):
    d = [0] * P
    for l, r in sched:
        d[l] = max(d[l], d[r]) + 1
    return max(d) if P > 1 else 0


@pytest.mark.parametrize("P", [1, 2, 3, 4, 7, 8, 256, 1023])
def test_tree_shapes(P):
    b = oracle.schedule(P, oracle.TREE_BINARY)
    assert len(b) == P - 1
    assert _depth(b, P) == (math.ceil(math.log2(P)) if P > 1 else 0)
    q = oracle.schedule(P, oracle.TREE_QUAD)
    assert len(q) == P - 1
    f = oracle.schedule(P, oracle.TREE_FLAT)
    assert f == [(0, i) for i in range(1, P)]
    for s in (b, q, f):     # every node is consumed once, results land left
        assert sorted(r for _, r in s) == list(range(1, P))


def test_paper_message_counts():
    """Fig. 2 caption: on an M x 3 matrix spread over three clusters the
    grid-tuned TSQR tree sends two inter-cluster messages, independent of the
    number of columns; Table 1: a binary tree over P domains has log2(P)
    messages on its critical path."""
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    for case in g["tuned_tree_inter_cluster"]:
        sizes = case["domains_per_cluster"]
        start = np.cumsum([0] + sizes[:-1]).tolist()
        sched = []
        for s0, sz in zip(start, sizes):            # binary tree inside a cluster
            sched += [(s0 + l, s0 + r) for l, r in oracle.schedule(sz, 2)]
        roots = start
        sched += [(roots[l], roots[r]) for l, r in oracle.schedule(len(roots), 2)]
        cluster = np.repeat(np.arange(len(sizes)), sizes)
        inter = sum(1 for l, r in sched if cluster[l] != cluster[r])
        assert inter == case["inter_cluster_messages"]
    for case in g["binary_tree_messages"]:
        P = case["P"]
        assert _depth(oracle.schedule(P, 2), P) == case["critical_path_messages"]


def test_hierarchical_schedule_inter_cluster_counts():
    """The grid-tuned tree builder: G - 1 combines join two clusters (the
    paper's inter-cluster message counts, Fig. 2 caption and Sec. 5), for
    contiguous clusters and for clusters interleaved the way domains fall
    on XCDs (domain d on cluster d mod G); every domain is combined into
    another exactly once, the root is domain 0, and the tree applied by the
    oracle gives the same R as the binary tree."""
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    for case in g["tuned_tree_inter_cluster"]:
        sizes = case["domains_per_cluster"]
        contiguous = np.repeat(np.arange(len(sizes)), sizes).tolist()
        P = len(contiguous)
        rng = np.random.default_rng(P)
        shuffled = rng.permutation(contiguous).tolist()
        for group in (contiguous, shuffled):
            sched = oracle.hierarchical_schedule(group)
            assert sum(1 for l, r in sched if group[l] != group[r]) == case["inter_cluster_messages"]
            assert sorted(r for _, r in sched) == [d for d in range(P) if d != 0]
    for P in (1, 3, 8, 9, 64, 256):
        group = [d % oracle.XCDS for d in range(P)]
        sched = oracle.hierarchical_schedule(group)
        assert sum(1 for l, r in sched if group[l] != group[r]) == min(P, oracle.XCDS) - 1
    A = np.random.default_rng(3).standard_normal((9000, 12))
    P = len(oracle.partition(9000, 12, 500))
    R1 = oracle.TSQR(A, mb=500, sched=oracle.hierarchical_schedule([d % 8 for d in range(P)])).R()
    R2 = oracle.TSQR(A, mb=500).R()
    assert rel(R1, R2) <= 1e-13


# ------------------------------------------------------------- whole TSQR

def test_single_domain_is_unpartitioned_householder():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((3000, 20))
    f = oracle.TSQR(A, mb=3000)
    assert f.P == 1
    R = f.R()
    assert rel(R, signfix(np.linalg.qr(A)[1])) <= 1e-14
    W, tau, _ = f.leaf()
    la, ltau, _, info = lapack.dgeqrf(np.asfortranarray(A.copy()))
    assert rel(tau, ltau) <= 1e-13


@pytest.mark.parametrize("m,n,mb", [(4096, 16, 1024), (5003, 13, 700), (2000, 40, 64), (777, 1, 100)])
def test_r_invariants_and_tree_independence(m, n, mb):
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    Rs = []
    for tree in (oracle.TREE_BINARY, oracle.TREE_QUAD, oracle.TREE_FLAT, 3):
        f = oracle.TSQR(A, mb=mb, tree=tree)
        R = f.R()
        assert np.all(np.tril(R, -1) == 0.0)
        assert np.all(np.diag(R) >= 0.0)
        assert np.linalg.norm(R.T @ R - A.T @ A) <= 64 * U * math.sqrt(m) * np.linalg.norm(A) ** 2
        Rs.append(R)
    # a shuffled pairing order is a valid tree too (commutativity, Sec. 2.3)
    P = len(oracle.partition(m, n, mb))
    order = [0] + (1 + rng.permutation(P - 1)).tolist()   # root stays slot 0
    sched = []
    live = order[:]
    while len(live) > 1:
        nxt = []
        for i in range(0, len(live) - 1, 2):
            a, b = live[i], live[i + 1]
            sched.append((a, b))
            nxt.append(a)
        if len(live) % 2:
            nxt.append(live[-1])
        live = nxt
    assert live[0] == 0
    f = oracle.TSQR(A, mb=mb, sched=sched)
    Rs.append(f.R())
    Rref = signfix(np.linalg.qr(A)[1])
    for R in Rs:
        assert rel(R, Rref) <= 1e-13


def test_shuffled_order_with_root_zero():
    rng = np.random.default_rng(42)
    A = rng.standard_normal((6400, 12))
    P = len(oracle.partition(6400, 12, 400))
    order = [0] + (1 + rng.permutation(P - 1)).tolist()
    sched = [(0, o) for o in order[1:]]        # flat tree, shuffled order
    R1 = oracle.TSQR(A, mb=400, sched=sched).R()
    R2 = oracle.TSQR(A, mb=400).R()
    assert rel(R1, R2) <= 1e-13


def _shuffled_binary_schedule(P, rng):
    """A binary tree over a random leaf order whose root is domain 0."""
    order = [0] + (1 + rng.permutation(P - 1)).tolist()
    sched, live = [], order[:]
    while len(live) > 1:
        nxt = []
        for i in range(0, len(live) - 1, 2):
            sched.append((live[i], live[i + 1]))
            nxt.append(live[i])
        if len(live) % 2:
            nxt.append(live[-1])
        live = nxt
    return sched


# (m, n, mb, tree): the binary, flat and 4-ary trees of Sec. 2.3, plus an
# explicit schedule (a binary tree over a shuffled leaf order, "shuffled");
# each with a ragged last domain in some cases.  Q and Q^T B follow the
# factorization's tree, so every traversal is pinned to NumPy's QR.
QSHAPES = [(4096, 16, 1024, 2), (5003, 13, 700, 2), (300, 30, 60, 2),
           (5003, 13, 700, 0), (4096, 16, 512, 0), (300, 30, 60, 0),
           (5003, 13, 700, 4), (9000, 20, 500, 4), (300, 30, 60, 4),
           (7001, 11, 600, "shuffled"), (3000, 25, 100, "shuffled")]


@pytest.mark.parametrize("m,n,mb,tree", QSHAPES)
def test_form_q_and_apply_qt(m, n, mb, tree):
    rng = np.random.default_rng(7 * m + n)
    A = rng.standard_normal((m, n))
    if tree == "shuffled":
        P = len(oracle.partition(m, n, mb))
        f = oracle.TSQR(A, mb=mb, sched=_shuffled_binary_schedule(P, rng))
    else:
        f = oracle.TSQR(A, mb=mb, tree=tree)
    Q, R = f.form_q(), f.R()
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13
    assert rel(Q @ R, A) <= 1e-13
    Qn, Rn = np.linalg.qr(A)
    d = np.where(np.diag(Rn) < 0, -1.0, 1.0)
    assert rel(Q, Qn * d) <= 1e-12
    B = rng.standard_normal((m, 3))
    C = f.apply_qt(B)
    assert rel(C[:n], Q.T @ B) <= 1e-13
    tail_expected = np.linalg.norm(B - Q @ (Q.T @ B), axis=0)
    assert np.allclose(np.linalg.norm(C[n:], axis=0), tail_expected, rtol=1e-12)
    # Q^T is orthogonal: column norms are preserved
    assert np.allclose(np.linalg.norm(C, axis=0), np.linalg.norm(B, axis=0), rtol=1e-13)
    # column by column: no small column of Q or Q^T B hides under a large one
    for j in range(n):
        assert np.linalg.norm(Q[:, j] - Qn[:, j] * d[j]) <= 1e-12
    QtB = Q.T @ B
    for c in range(3):
        assert np.linalg.norm(C[:n, c] - QtB[:, c]) <= 1e-13 * np.linalg.norm(B[:, c])


def test_lsq_against_lapack_and_consistent_rhs():
    rng = np.random.default_rng(9)
    m, n = 5000, 24
    A = rng.standard_normal((m, n))
    f = oracle.TSQR(A, mb=800)
    B = rng.standard_normal((m, 2))
    X, res, info = f.lsq(B)
    assert info == 0
    _, Xl, _ = lapack.dgels(np.asfortranarray(A.copy()), np.asfortranarray(B.copy()))[:3]
    Xl = Xl[:n]
    kappa = np.linalg.cond(A)
    tan = np.linalg.norm(B - A @ Xl, axis=0) / np.linalg.norm(A @ Xl, axis=0)
    kls = kappa + kappa ** 2 * tan
    for c in range(2):
        assert rel(X[:, c], Xl[:, c]) <= 10 * kls[c] * U
        assert abs(res[c] - np.linalg.norm(B[:, c] - A @ X[:, c])) <= 1e-12 * res[c]
        r = B[:, c] - A @ X[:, c]
        eta = np.linalg.norm(A.T @ r) / (np.linalg.norm(A) * (np.linalg.norm(A) * np.linalg.norm(X[:, c]) + np.linalg.norm(B[:, c])))
        assert eta <= 1e-14
    xt = rng.standard_normal(n)
    Xc, res_c, _ = f.lsq(A @ xt)
    assert rel(Xc[:, 0], xt) <= 10 * kappa * U * math.sqrt(n)
    assert res_c[0] <= 1e-13 * np.linalg.norm(A @ xt)


# --------------------------------------------- exact rational brute force

def _exact_checks(A, R, tol_rel=16 * U):
    """R^T R = A^T A in exact rationals, entry by entry, with the floating R
    converted exactly; tolerance relative to ||A||_F^2."""
    Af = [[Fraction(float(x)) for x in row] for row in A]
    Rf = [[Fraction(float(x)) for x in row] for row in R]
    m, n = len(Af), len(Af[0])
    nrm2 = sum(x * x for row in Af for x in row)
    for i in range(n):
        for j in range(n):
            g = sum(Af[r][i] * Af[r][j] for r in range(m))
            h = sum(Rf[q][i] * Rf[q][j] for q in range(n))
            if abs(float(g - h)) > tol_rel * float(nrm2):
                return False
    return True


@pytest.mark.parametrize("mb", [2, 4])
def test_brute_force_4x2_closed_form(mb):
    rng = np.random.default_rng(123)
    for _ in range(200):
        A = rng.standard_normal((4, 2))
        R = oracle.TSQR(A, mb=mb).R()
        a1 = [Fraction(float(x)) for x in A[:, 0]]
        a2 = [Fraction(float(x)) for x in A[:, 1]]
        n11 = sum(x * x for x in a1)
        n12 = sum(x * y for x, y in zip(a1, a2))
        n22 = sum(x * x for x in a2)
        r11, r12, r22 = (Fraction(float(R[0, 0])), Fraction(float(R[0, 1])), Fraction(float(R[1, 1])))
        assert abs(float(r11 * r11 - n11)) <= 16 * U * float(n11)
        assert abs(float(r11 * r12 - n12)) <= 16 * U * float(n11 + n22)
        exact22 = n22 - n12 * n12 / n11
        assert abs(float(r22 * r22 - exact22)) <= 16 * U * float(n11 + n22)


def test_brute_force_integer_4x2_enumeration():
    """A deterministic subset of the 5^8 integer matrices with entries in
    {-2..2}; every full-rank one must give R^T R = A^T A exactly up to 16u."""
    vals = [-2, -1, 0, 1, 2]
    count = 0
    for idx in range(0, 5 ** 8, 97):      # every 97th matrix: ~4000 cases
        digits = []
        t = idx
        for _ in range(8):
            digits.append(vals[t % 5])
            t //= 5
        A = np.array(digits, dtype=np.float64).reshape(4, 2)
        if abs(np.linalg.det(A.T @ A)) < 0.5:   # integer Gram: singular iff det 0
            continue
        for mb in (2, 4):
            R = oracle.TSQR(A, mb=mb).R()
            assert _exact_checks(A, R)
        count += 1
    assert count > 3000


@pytest.mark.parametrize("shape,mb", [((8, 2), 2), ((8, 2), 4), ((8, 4), 4), ((8, 4), 8)])
def test_brute_force_8_rows(shape, mb):
    rng = np.random.default_rng(shape[1] * 10 + mb)
    for _ in range(50):
        A = rng.standard_normal(shape)
        f = oracle.TSQR(A, mb=mb)
        assert f.P == shape[0] // mb
        assert _exact_checks(A, f.R())


# ------------------------------------------------- closed forms / specials

def test_single_column_closed_form():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((1000, 1))
    f = oracle.TSQR(a, mb=128)
    assert abs(f.R()[0, 0] - np.linalg.norm(a)) <= 8 * U * np.linalg.norm(a)
    assert rel(f.form_q(), a / np.linalg.norm(a)) <= 16 * U * math.sqrt(1000)


def test_orthonormal_input_gives_identity_and_triangular_input_gives_itself():
    rng = np.random.default_rng(4)
    Q0 = np.linalg.qr(rng.standard_normal((2048, 10)))[0]
    assert np.linalg.norm(oracle.TSQR(Q0, mb=256).R() - np.eye(10)) <= 1e-14
    R0 = np.triu(rng.standard_normal((10, 10))) + 5 * np.eye(10)
    R0 = signfix(R0)
    assert rel(oracle.TSQR(Q0 @ R0, mb=256).R(), R0) <= 1e-13


def test_power_of_two_column_scaling_is_exact():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((3000, 9))
    d = 2.0 ** rng.integers(-20, 20, size=9)
    R = oracle.TSQR(A, mb=500).R()
    Rd = oracle.TSQR(A * d, mb=500).R()
    assert np.array_equal(Rd, R * d)


def test_row_permutation_invariance_and_square_case():
    rng = np.random.default_rng(10)
    A = rng.standard_normal((1200, 15))
    p = rng.permutation(1200)
    assert rel(oracle.TSQR(A[p], mb=300).R(), oracle.TSQR(A, mb=300).R()) <= 1e-13
    S = rng.standard_normal((15, 15))
    f = oracle.TSQR(S, mb=15)
    assert rel(f.form_q() @ f.R(), S) <= 1e-14


def test_exact_zero_column():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((2000, 6))
    A[:, 3] = 0.0
    f = oracle.TSQR(A, mb=400)
    R = f.R()
    assert R[3, 3] == 0.0
    W, tau, T = f.leaf()
    assert np.all(tau[:, 3] == 0.0)
    _, _, info = f.lsq(rng.standard_normal(2000))
    assert info == 4


def test_conditioned_construction_singular_values():
    """A = U diag(s) V^T: the singular values of R equal s (closed form from
    the construction), checked at a reduced row count."""
    def orth(G):
        return oracle.TSQR(G, mb=max(G.shape[1], 4096)).form_q()
    A, b, bc, xt, s = synth.config_conditioned(16384, 128, orth, seed=0)
    f = oracle.TSQR(A, mb=4096)
    sv = np.linalg.svd(f.R(), compute_uv=False)
    assert np.max(np.abs(sv - s)) <= 200 * U * math.sqrt(16384) * np.linalg.norm(A, 2)


def test_refined_reference_converges_on_ill_conditioned_lsq():
    rng = np.random.default_rng(13)
    m, n = 6000, 20
    Uq = np.linalg.qr(rng.standard_normal((m, n)))[0]
    Vq = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = synth.log_spaced_spectrum(n, -6)
    A = (Uq * s) @ Vq.T
    b = rng.standard_normal(m)
    f = oracle.TSQR(A, mb=1000)
    x, it = f.lsq_refined(A, b)
    assert it >= 1
    # normal equations hold to the accuracy of the data
    r = b - A @ x
    eta = np.linalg.norm(A.T @ r) / (np.linalg.norm(A) * (np.linalg.norm(A) * np.linalg.norm(x) + np.linalg.norm(b)))
    assert eta <= 1e-15


# ------------------------------------------------- block orthogonalisation

@pytest.mark.parametrize("m,nv,b,mb", [(5000, 0, 8, 1000), (5000, 24, 8, 1000), (3001, 40, 13, 700),
                                       (2000, 100, 32, 512)])
def test_block_orth_invariants(m, nv, b, mb):
    """The oracle's block orthogonalisation step against what the
    mathematics fixes: [V Q] orthonormal, W = V H + Q R, R upper triangular
    with diag >= 0, H = V^T W (exactly in exact arithmetic, since V^T (W - V H1)
    = 0 for orthonormal V), and with no basis it is plain TSQR."""
    rng = np.random.default_rng(m + nv + b)
    V = np.linalg.qr(rng.standard_normal((m, nv)))[0] if nv else None
    W = rng.standard_normal((m, b))
    Q, H, R = oracle.block_orth(V, W, mb)
    B = Q if V is None else np.hstack([V, Q])
    assert np.linalg.norm(B.T @ B - np.eye(B.shape[1])) <= 1e-13
    recon = Q @ R if V is None else V @ H + Q @ R
    assert rel(recon, W) <= 1e-14
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
    if V is not None:
        assert rel(H, V.T @ W) <= 1e-14
    else:
        assert rel(R, oracle.TSQR(W, mb=mb).R()) == 0.0


def test_block_orth_of_a_block_in_the_complement():
    """A block already orthogonal to V has H = 0 and Q R = W; a block inside
    span(V) plus a small complement keeps orthogonality to V (the second
    pass), the case a single Gram-Schmidt pass gets wrong."""
    rng = np.random.default_rng(5)
    m, nv, b = 4000, 30, 6
    V = np.linalg.qr(rng.standard_normal((m, nv)))[0]
    G = rng.standard_normal((m, b))
    W = G - V @ (V.T @ G)
    Q, H, R = oracle.block_orth(V, W, 800)
    assert np.linalg.norm(H) <= 1e-14 * np.linalg.norm(W)
    assert rel(Q @ R, W) <= 1e-14
    W2 = V @ rng.standard_normal((nv, b)) + 1e-8 * G
    Q2, H2, R2 = oracle.block_orth(V, W2, 800)
    assert np.linalg.norm(V.T @ Q2) <= 1e-13
    assert rel(V @ H2 + Q2 @ R2, W2) <= 1e-14



# ---------------------------------------------------------------- Cholesky

def test_cholesky_pascal_closed_form():
    # The symmetric Pascal matrix S_ij = C(i + j, i) has the lower Pascal
    # matrix L_ij = C(i, j) as its Cholesky factor (a unit diagonal, so every
    # step is integer arithmetic, exact in FP64 while the entries stay below
    # 2^53).  A dropped term, a transposed index or a wrong sign changes some
    # binomial.
    n = 20
    S = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    L, info = oracle.cholesky(S)
    assert info == 0
    want = np.array([[math.comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)], dtype=np.float64)
    assert np.array_equal(L, want)


def test_cholesky_small_closed_forms():
    L, info = oracle.cholesky(np.array([[9.0]]))
    assert info == 0 and L[0, 0] == 3.0
    L, info = oracle.cholesky(np.array([[4.0, 2.0], [2.0, 5.0]]))
    assert info == 0 and np.array_equal(L, np.array([[2.0, 0.0], [1.0, 2.0]]))
    # 3 x 3 with L = [[2,0,0],[6,1,0],[-8,5,3]] (a textbook example)
    Lw = np.array([[2.0, 0, 0], [6, 1, 0], [-8, 5, 3]])
    L, info = oracle.cholesky(Lw @ Lw.T)
    assert info == 0 and np.array_equal(L, Lw)


@pytest.mark.parametrize("n", [1, 7, 50, 130])
def test_cholesky_backward_error_and_lapack(n):
    A = synth.spd_gram(n, seed=300 + n)
    L, info = oracle.cholesky(A)
    assert info == 0
    assert np.array_equal(L, np.tril(L)) and np.all(np.diag(L) > 0)
    # backward stability: L L^T = A + E with |E| <= gamma_{n+1} |L| |L^T|
    E = np.abs(L @ L.T - A)
    bound = (n + 1) * U / (1 - (n + 1) * U) * (np.abs(L) @ np.abs(L.T))
    assert np.all(E <= 2.0 * bound + 1e-300)
    # LAPACK's dpotrf (through SciPy) factors the same matrix: kappa ~ 34
    Ll = scipy.linalg.cholesky(A, lower=True)
    assert np.max(np.abs(L - Ll)) <= 64 * n * U * 34 * np.max(np.abs(Ll))


def test_cholesky_reads_lower_triangle_only():
    n = 40
    A = synth.spd_gram(n, seed=7)
    B = A.copy(order="F")
    B[np.triu_indices(n, 1)] = np.random.default_rng(8).standard_normal(n * (n - 1) // 2) * 1e3
    assert np.array_equal(oracle.cholesky(A)[0], oracle.cholesky(B)[0])


def test_cholesky_power_of_two_scaling_is_exact():
    # chol(D A D) = D chol(A) for D = diag(2^e_i): every operation scales by
    # an exact power of two.
    n = 60
    A = synth.spd_gram(n, seed=9)
    e = np.random.default_rng(10).integers(-30, 31, n)
    D = np.ldexp(1.0, e)
    L, info = oracle.cholesky(D[:, None] * A * D[None, :])
    L0, _ = oracle.cholesky(A)
    assert info == 0 and np.array_equal(L, D[:, None] * L0)


def test_cholesky_info_on_indefinite_and_singular():
    # diag(1, 1, -1, 1): the leading minor of order 3 is negative
    L, info = oracle.cholesky(np.diag([1.0, 1.0, -1.0, 1.0]))
    assert info == 3
    assert np.array_equal(L[:, :2], np.eye(4)[:, :2]) and not L[:, 2:].any()
    # a singular leading 2 x 2 block: the second pivot is exactly zero
    L, info = oracle.cholesky(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    assert info == 2 and L[0, 0] == 1.0 and L[1, 0] == 1.0
    # a NaN on the diagonal fails at once
    A = synth.spd_gram(5, seed=1)
    A[0, 0] = np.nan
    assert oracle.cholesky(A)[1] == 1
    # a rank-deficient Gram matrix (k < n) fails somewhere past column k
    A = synth.spd_gram(30, seed=2, k=10)
    assert oracle.cholesky(A)[1] > 10


# ---------------------------------------------------------------- CALU

def _calu_parts(LU, ipiv):
    m, n = LU.shape
    L = np.tril(LU, -1)[:, :n] + np.eye(m, n)
    U = np.triu(LU[:n, :])
    perm = np.arange(m)
    for i, p in enumerate(ipiv):
        perm[[i, p]] = perm[[p, i]]
    return L, U, perm


@pytest.mark.parametrize("m,n", [(5, 5), (64, 64), (100, 100), (200, 64), (256, 130), (130, 70), (90, 1)])
def test_calu_is_lapack_getrf_when_one_stack_holds_each_panel(m, n):
    # m <= 256: every panel's tournament is one stack, i.e. Gaussian
    # elimination with partial pivoting, so the pivots are LAPACK's dgetrf's
    # exactly and the factors agree to rounding
    A = synth.gaussian(m, n, seed=600 + m + n)
    LU, ipiv, info = oracle.calu(A, mb=4096)
    lu, piv = scipy.linalg.lu_factor(A)
    assert info == 0
    assert ipiv.tolist() == piv.tolist()
    assert np.max(np.abs(LU - lu)) <= 1e-12 * max(1.0, np.abs(lu).max())


@pytest.mark.parametrize("m,n,mb,tree", [(3000, 200, 512, oracle.TREE_BINARY), (2500, 130, 600, oracle.TREE_QUAD),
                                         (1500, 64, 256, oracle.TREE_FLAT), (800, 800, 300, oracle.TREE_BINARY)])
def test_calu_reconstructs_a_and_keeps_multipliers_bounded(m, n, mb, tree):
    A = synth.gaussian(m, n, seed=7 + m)
    LU, ipiv, info = oracle.calu(A, mb=mb, tree=tree)
    assert info == 0
    L, U, perm = _calu_parts(LU, ipiv)
    assert sorted(perm.tolist()) == list(range(m))
    assert np.all(ipiv >= np.arange(n)) and np.all(ipiv < m)
    res = np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A)
    assert res <= 1e-14 * np.sqrt(n)
    # tournament pivoting keeps the multipliers small (|l| = 1 only for
    # partial pivoting; the tournament's bound is looser but far from growth)
    assert np.abs(L).max() <= 16.0


def test_calu_single_column_is_the_argmax():
    A = synth.gaussian(5000, 1, seed=3)
    LU, ipiv, info = oracle.calu(A, mb=700)
    p = int(np.argmax(np.abs(A[:, 0])))
    assert info == 0 and ipiv[0] == p
    assert LU[0, 0] == A[p, 0]
    rest = np.delete(np.arange(5000), [p])
    # row p came to the top; the old top row went to position p
    col = A[:, 0].copy()
    col[[0, p]] = col[[p, 0]]
    assert np.array_equal(LU[1:, 0], col[1:] / A[p, 0])


def test_calu_zero_column_sets_info_and_goes_on():
    A = synth.gaussian(400, 100, seed=4)
    A[:, 70] = 0.0
    LU, ipiv, info = oracle.calu(A, mb=128)
    assert info == 71
    L, U, perm = _calu_parts(LU, ipiv)
    assert U[70, 70] == 0.0 and not np.tril(LU, -1)[:, 70].any()
    assert np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A) <= 1e-14 * 10
