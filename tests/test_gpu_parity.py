"""GPU parity: the HIP library against the FP64 CPU oracle, element by
element on the same seeded inputs.

Tolerances (the FP64 accuracy targets of the least-squares workloads):
  R:   ||R_gpu - R_oracle||_F / ||R_oracle||_F <= 1e-12 after both are
       sign-normalised (R with diag >= 0 is unique, Sec. 2.2);
  Q:   ||A - Q R||_F / ||A||_F <= 1e-13 and ||Q^T Q - I||_F <= 1e-13;
       Q itself is unique once R is, so it is compared to the oracle's Q;
  Q^T B: rows 0..n-1 equal Q_1^T B (unique); rows n..m-1 depend on the
       representation, so only their column norms are compared;
  least squares: x unique for full-rank A; compared within
       max(1e-12, 10 kappa_LS u).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def tl():
    import paper_0912_2572_amd as t
    t.lib()
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return t


def dev(x):
    t = torch.as_tensor(np.asarray(x, dtype=np.float64))
    if t.dim() == 2:
        t = t.t().contiguous().t()
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def colwise(a, b, tol, scale=None):
    """Column by column: ||a_j - b_j|| <= tol * (scale_j or ||b_j||), so a
    wrong small column cannot hide under a large one in a Frobenius norm."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    for j in range(b.shape[1]):
        ref = np.linalg.norm(b[:, j]) if scale is None else scale[j]
        err = np.linalg.norm(a[:, j] - b[:, j])
        assert err <= tol * max(ref, 1e-300), f"column {j}: {err:.3e} > {tol:.1e} * {ref:.3e}"


def r_entrywise(R, Ro, tol=1e-12):
    """Every entry of R within tol of its column's norm (R_ij is a dot of
    column j of A with a unit vector, so |error| scales with ||a_j||)."""
    cn = np.linalg.norm(Ro, axis=0)
    assert np.all(np.abs(R - Ro) <= tol * np.maximum(cn, 1e-300)[None, :]), \
        float(np.max(np.abs(R - Ro) / np.maximum(cn, 1e-300)[None, :]))


def check_all(tl, A, mb, tree=2, nrhs=2, seed=0, full_q=True, domains=0, weights=None):
    m, n = A.shape
    print(f"case m={m} n={n} mb={mb} tree={tree} domains={domains} weights={weights is not None}", flush=True)
    if domains or weights is not None:
        # the load-balanced or weighted partition: the oracle factors over the
        # library's domains, which must be its own apportionment
        po = tl.opts(domains=domains) if domains else tl.opts(weights=weights)
        parts = tl.partition(m, n, po)
        P, chunk, _ = tl.plan_info(m, n, po)
        assert parts == oracle.partition_weighted(m, n, P, chunk, weights)
        sched = tl.tree_schedule(P, tree) if tree == tl.TREE_XCD else None
        orc = oracle.TSQR(A, parts=parts, tree=tree, sched=sched)
    elif tree == tl.TREE_XCD:
        # the oracle runs the hierarchical schedule over its own domains (for
        # n > 64 the GPU's first panel merges a short last domain by its own
        # width, so the counts can differ; R, Q and x do not depend on it)
        P = len(oracle.partition(m, n, mb))
        sched = tl.tree_schedule(P, tree)
        assert sorted(sched) == sorted(oracle.hierarchical_schedule([d % 8 for d in range(P)]))
        orc = oracle.TSQR(A, mb=mb, sched=sched)
    else:
        orc = oracle.TSQR(A, mb=mb, tree=tree)
    Ad = dev(A)
    if weights is not None:
        f = tl.factor(Ad, weights=weights, tree=tree)
    elif domains:
        f = tl.factor(Ad, domains=domains, tree=tree)
    else:
        f = tl.factor(Ad, row_block=mb, tree=tree)
    R = host(f.R())
    Ro = orc.R()
    assert np.all(np.tril(R, -1) == 0.0)
    assert np.all(np.diag(R) >= 0.0)
    assert rel(R, Ro) <= 1e-12
    r_entrywise(R, Ro)
    if full_q:
        Q = host(f.form_q())
        assert rel(Q @ R, A) <= 1e-13
        assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13
        Qo = orc.form_q()
        assert rel(Q, Qo) <= 1e-12
        colwise(Q, Qo, 1e-12)
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, nrhs))
    Bd = dev(B)
    f.apply_qt_(Bd)
    C = host(Bd)
    Co = orc.apply_qt(B)
    assert rel(C[:n], Co[:n]) <= 1e-12
    colwise(C[:n], Co[:n], 1e-12, scale=np.linalg.norm(B, axis=0))
    assert np.allclose(np.linalg.norm(C[n:], axis=0), np.linalg.norm(Co[n:], axis=0), rtol=1e-11,
                       atol=1e-13 * np.linalg.norm(B))
    f.apply_q_(Bd)
    assert rel(host(Bd), B) <= 1e-13
    X, res, info = f.lsq(dev(B))
    torch.cuda.synchronize()
    Xo, reso, infoo = orc.lsq(B)
    assert int(info.item()) == infoo == 0
    kappa = np.linalg.cond(Ro)
    for c in range(nrhs):
        tan = reso[c] / max(np.linalg.norm(A @ Xo[:, c]), 1e-300)
        tol = max(1e-12, 10 * (kappa + kappa ** 2 * tan) * U)
        assert rel(host(X)[:, c], Xo[:, c]) <= tol
        # entry by entry: x_i = e_i^T R^{-1} c, so each entry's error is
        # bounded by the same relative tolerance times ||x||
        assert np.max(np.abs(host(X)[:, c] - Xo[:, c])) <= tol * np.linalg.norm(Xo[:, c])
    assert np.allclose(host(res), reso, rtol=1e-11)
    return f


def test_small_config(tl):
    """4096 x 16, N(0,1) from seed 0, four 1024-row domains, binary tree,
    R, implicit Q and the least-squares solution of one b ~ N(0,1)."""
    A, b = synth.config_small(0)
    f = check_all(tl, A, 1024, 2, nrhs=1)
    X, res, info = f.lsq(dev(b.reshape(-1, 1)))
    xo, reso, _ = oracle.TSQR(A, mb=1024).lsq(b)
    assert rel(host(X)[:, 0], xo[:, 0]) <= 1e-12
    assert abs(host(res)[0] - reso[0]) <= 1e-12 * reso[0]


SHAPES = [
    # (m, n, mb, tree): ragged domains and chunks, several tiles per chunk,
    # every slot width (n <= 8, 16, 32, 64), every tree
    (64, 64, 64, 2),
    (65, 64, 64, 2),
    (1000, 3, 100, 2),
    (1000, 1, 128, 0),
    (1023, 17, 256, 4),
    (4097, 32, 512, 2),
    (4097, 32, 512, 0),
    (10000, 2, 2048, 4),
    (65537, 8, 4096, 2),
    (20000, 64, 1500, 2),
    (20000, 64, 3000, 4),
    (9000, 40, 700, 0),
    (3000, 33, 300, 2),
    # even m (16-byte aligned reflector columns: half of each full chunk's
    # reflectors leave through LDS during the next chunk), n < 64, long runs
    # of full chunks, the drain after a domain's last chunk and into a tail
    (40000, 48, 4096, 2),
    (50002, 40, 2048, 4),
    # the hierarchical (XCD) tree: P below, at and above the 8 XCDs, ragged
    (5000, 16, 1024, 8),
    (65536, 64, 4096, 8),
    (100003, 33, 1024, 8),
    (300000, 8, 2048, 8),
]


@pytest.mark.parametrize("m,n,mb,tree", SHAPES)
def test_shapes(tl, m, n, mb, tree):
    A = synth.gaussian(m, n, seed=m + n)
    check_all(tl, A, mb, tree)


# (m, n, domains, tree): the load-balanced partition (opts.domains, Sec. 3):
# one domain per compute unit with a remainder of chunks spread over the
# first domains, the narrow leaves' two per unit (-1), every tree, a tiny
# ragged case and two 64-column panels balanced one by one
BALANCED_SHAPES = [
    (300_000, 64, 256, 2),
    (100_003, 20, -1, 2),
    (70_001, 32, 300, 4),
    (50_000, 48, 100, 0),
    (200_000, 8, 256, 8),
    (5003, 13, 7, 2),
    (20_000, 100, 16, 2),
]


@pytest.mark.parametrize("m,n,domains,tree", BALANCED_SHAPES)
def test_balanced_domains(tl, m, n, domains, tree):
    A = synth.gaussian(m, n, seed=m + 3 * n)
    check_all(tl, A, 0, tree, domains=domains)


# (m, n, weights, tree): rows in proportion to per-domain powers (Sec. 3)
WEIGHTED_SHAPES = [
    (300_000, 64, [1, 2, 3, 4] * 64, 2),
    (100_003, 20, [3, 1] * 50, 4),
    (50_000, 48, [5, 1, 2, 7, 3], 0),
    (200_000, 8, [2, 1, 1, 1] * 16, 8),
    (20_000, 100, [1, 2, 3], 2),
]


@pytest.mark.parametrize("m,n,weights,tree", WEIGHTED_SHAPES)
def test_weighted_domains(tl, m, n, weights, tree):
    A = synth.gaussian(m, n, seed=m + 5 * n)
    check_all(tl, A, 0, tree, weights=weights)


def test_weighted_domains_factor_solve_and_tslu(tl):
    """tsqr_factor_solve (the forked FP64 schedule) and TSLU over weighted
    domains against the oracle on the same domains."""
    m, n = 150_001, 64
    w = [3, 1] * 64
    print(f"case weighted factor_solve and TSLU m={m} n={n}", flush=True)
    A = synth.gaussian(m, n, seed=51)
    b = np.random.default_rng(52).standard_normal((m, 1))
    o = tl.opts(weights=w, lsq_max_rhs=1)
    Q = tl.empty_colmajor(m, n, device="cuda")
    F, X, r, info = tl.factor_solve(dev(A), dev(b), o, Q=Q)
    torch.cuda.synchronize()
    parts = tl.partition(m, n, o)
    orc = oracle.TSQR(A, parts=parts)
    xo, ro, _ = orc.lsq(b)
    assert int(info.item()) == 0
    colwise(host(X), xo, 1e-12, scale=np.linalg.norm(xo, axis=0))
    colwise(host(Q), orc.form_q(), 1e-12)
    r_entrywise(host(F.R()), orc.R())
    ipiv, L, U, linfo = tl.tslu(dev(A), o)
    torch.cuda.synchronize()
    ipo, Lo, Uo, _ = oracle.tslu(A, parts, first=256, stage=256 - n)
    assert host(ipiv).tolist() == ipo.tolist()
    assert np.max(np.abs(host(U) - Uo)) <= 1e-13 * np.abs(Uo).max()
    assert np.max(np.abs(host(L) - Lo)) <= 1e-12 * max(1.0, np.abs(Lo).max())


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_balanced_domains_factor_solve(tl, prec):
    """tsqr_factor_solve over balanced domains (the forked FP64 schedule, or
    the mixed path's refinement) against the oracle's solution."""
    m, n, domains = 150_001, 64, 256
    print(f"case balanced factor_solve m={m} n={n} domains={domains} {prec}", flush=True)
    A = synth.gaussian(m, n, seed=41)
    b = np.random.default_rng(42).standard_normal((m, 1))
    o = tl.opts(domains=domains, lsq_max_rhs=1, prec=tl.MIXED if prec == "mixed" else tl.F64)
    Q = tl.empty_colmajor(m, n, device="cuda")
    F, X, r, info = tl.factor_solve(dev(A), dev(b), o, Q=Q)
    torch.cuda.synchronize()
    parts = tl.partition(m, n, o)
    orc = oracle.TSQR(A, parts=parts)
    xo, ro, _ = orc.lsq(b)
    assert int(info.item()) == 0
    colwise(host(X), xo, 1e-12, scale=np.linalg.norm(xo, axis=0))
    assert abs(host(r)[0] - ro[0]) <= 1e-11 * ro[0]
    Qh = host(Q)
    assert np.linalg.norm(Qh.T @ Qh - np.eye(n)) <= (1e-13 if prec == "f64" else 1e-5)
    if prec == "f64":
        colwise(Qh, orc.form_q(), 1e-12)
    r_entrywise(host(F.R()), orc.R())


@pytest.mark.parametrize("scale_exp", [-400, -250, 400])
def test_extreme_scales(tl, scale_exp):
    """Entries at the ends of the supported magnitudes, 2^-400 and 2^400
    (sums of squares near 2^-800 and 2^800, the range the Householder
    scalars' reciprocal square root covers), and in between: R, Q and x
    against the oracle (plain FP64 sums, as the paper's norms)."""
    m, n, mb = 20000, 64, 4096
    print(f"case scale 2^{scale_exp}", flush=True)
    A = np.ldexp(synth.gaussian(m, n, seed=77), scale_exp)
    check_all(tl, A, mb, 2, nrhs=1)


def strided_view(A, row_off, extra_rows):
    """A as a view into a taller column-major device matrix: leading
    dimension m + extra_rows, first row at row_off (row_off odd: the view's
    columns start off 16-byte boundaries)."""
    m, n = A.shape
    big = np.zeros((m + extra_rows, n))
    big[row_off:row_off + m] = A
    Bd = dev(big)
    return Bd[row_off:row_off + m]


@pytest.mark.parametrize("m,n,mb,row_off,extra", [
    (10001, 24, 1001, 0, 0),     # odd row block: 8-byte loads for every chunk
    (9000, 64, 2049, 0, 0),      # odd row block, wide kernel
    (20000, 40, 2048, 0, 6),     # lda = m + 6 (even: 16-byte loads still allowed)
    (20000, 40, 2048, 3, 8),     # row offset 3: columns start off 16-byte boundaries
    (8193, 16, 1024, 1, 1),      # odd lda and odd offset, narrow kernel
])
def test_layouts(tl, m, n, mb, row_off, extra):
    """Odd row blocks, a leading dimension larger than m and a view of A
    that starts at an odd row (the leaf's 16-byte loads must fall back to
    8-byte loads wherever a chunk would not start on a 16-byte boundary)."""
    A = synth.gaussian(m, n, seed=m + n + row_off)
    print(f"case layout m={m} n={n} mb={mb} row_off={row_off} lda={m + extra}", flush=True)
    Ad = strided_view(A, row_off, extra)
    assert Ad.stride(1) == m + extra
    orc = oracle.TSQR(A, mb=mb)
    f = tl.factor(Ad, row_block=mb)
    R, Ro = host(f.R()), orc.R()
    assert rel(R, Ro) <= 1e-12
    r_entrywise(R, Ro)
    Q = host(f.form_q())
    Qo = orc.form_q()
    colwise(Q, Qo, 1e-12)
    b = np.random.default_rng(m).standard_normal((m, 1))
    X, res, info = f.lsq(dev(b))
    torch.cuda.synchronize()
    Xo, reso, _ = orc.lsq(b)
    assert int(info.item()) == 0
    assert rel(host(X), Xo) <= 1e-12


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_nonfinite_input_info(tl, bad, prec):
    """A NaN or an infinity in A: the factor completes (no pivoting, no
    data-dependent loop), and the least-squares solve reports the documented
    dinfo = -2 (non-finite residual)."""
    m, n = 6000, 20
    A = synth.gaussian(m, n, seed=77)
    A[4321, 5] = bad
    print(f"case non-finite A ({bad}, {prec})", flush=True)
    Ad = dev(A)
    f = tl.factor(Ad, row_block=1024, prec=tl.MIXED if prec == "mixed" else tl.F64)
    b = dev(np.ones((m, 1)))
    _, res, info = f.lsq(b, A=Ad)
    torch.cuda.synchronize()
    assert int(info.item()) == -2
    assert not np.isfinite(host(res)[0])


@pytest.mark.parametrize("m,n,mb,tree", [(5000, 65, 1024, 2), (3000, 128, 512, 2), (4096, 200, 1024, 2),
                                         (2048, 256, 512, 2), (40000, 100, 1024, 8),
                                         # past 256 columns (the 16-slot final solve), up to
                                         # square: 5 to 16 panels
                                         (20000, 300, 4096, 2), (8000, 512, 2048, 2), (5000, 777, 1024, 4),
                                         (1024, 1024, 1024, 2)])
def test_wide_panels(tl, m, n, mb, tree):
    A = synth.gaussian(m, n, seed=m * 3 + n)
    check_all(tl, A, mb, tree)


def test_zero_column_info(tl):
    A = synth.gaussian(3000, 12, seed=5)
    A[:, 7] = 0.0
    f = tl.factor(dev(A), row_block=500)
    R = host(f.R())
    assert R[7, 7] == 0.0
    assert rel(R, oracle.TSQR(A, mb=500).R()) <= 1e-12
    X0 = torch.full((12, 1), 7.0, dtype=torch.float64, device="cuda")
    X0 = X0.t().contiguous().t()
    _, _, info = f.lsq(dev(np.ones((3000, 1))), X=X0)
    torch.cuda.synchronize()
    assert int(info.item()) == 8
    assert torch.all(X0 == 7.0)


def test_form_q_concurrent_with_solve(tl):
    """The documented exception to call ordering: for an FP64 factor with
    n <= 64 the thin Q may be formed on another stream while the same factor
    solves a least-squares problem; both results equal (bitwise) those of
    the two calls made one after the other."""
    A = synth.gaussian(60000, 64, seed=21)
    b = np.random.default_rng(22).standard_normal((60000, 1))
    Ad, bd = dev(A), dev(b)
    print("case form_q || lsq, 60000 x 64", flush=True)
    f = tl.factor(Ad, row_block=4096, lsq_max_rhs=1)
    Q1 = f.form_q()
    X1, r1, _ = f.lsq(bd)
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    for rep in range(3):
        Q2 = torch.empty_like(Q1)
        X2 = torch.full_like(X1, -1.0)
        side.wait_stream(main)
        with torch.cuda.stream(side):
            f.form_q(Q2)
        _, r2, info = f.lsq(bd, X=X2)
        main.wait_stream(side)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert torch.equal(Q2, Q1), f"rep {rep}"
        assert torch.equal(X2, X1) and torch.equal(r2, r1), f"rep {rep}"


@pytest.mark.parametrize("m,n,mb,prec,k,with_q", [
    (60000, 64, 4096, "f64", 1, True),     # forked: leaf pass of Q^T b beside the tree
    (70001, 33, 2048, "f64", 2, False),    # forked, ragged last domain, no thin Q
    (20000, 100, 4096, "f64", 1, True),    # two panels: the three calls in order
    (40000, 48, 4096, "mixed", 1, True),   # mixed precision: the three calls in order
])
def test_factor_solve_matches_separate_calls(tl, m, n, mb, prec, k, with_q):
    """tsqr_factor_solve gives bitwise the results of tsqr_factor,
    tsqr_lsq_solve and tsqr_form_q called one after the other, also for two
    calls enqueued back to back (the second reuses the fork's events)."""
    print(f"case factor_solve m={m} n={n} mb={mb} {prec} k={k} q={with_q}", flush=True)
    A = synth.gaussian(m, n, seed=31)
    b = np.random.default_rng(32).standard_normal((m, k))
    Ad, bd = dev(A), dev(b)
    o = tl.opts(row_block=mb, lsq_max_rhs=k, prec=tl.MIXED if prec == "mixed" else tl.F64)
    f = tl.Factors(Ad, o)
    X1, r1, i1 = f.lsq(bd, A=Ad)
    Q1 = f.form_q() if with_q else None
    R1 = f.R()
    torch.cuda.synchronize()
    outs = []
    for rep in range(2):
        Q2 = tl.empty_colmajor(m, n, device=Ad.device) if with_q else None
        F, X2, r2, i2 = tl.factor_solve(Ad, bd, o, Q=Q2)
        outs.append((F, X2, r2, i2, Q2))
    torch.cuda.synchronize()
    for rep, (F, X2, r2, i2, Q2) in enumerate(outs):
        assert int(i2.item()) == int(i1.item()) == 0, f"rep {rep}"
        assert torch.equal(X2, X1) and torch.equal(r2, r1), f"rep {rep}"
        assert torch.equal(F.R(), R1), f"rep {rep}"
        if with_q:
            assert torch.equal(Q2, Q1), f"rep {rep}"
    # the handle serves later calls like one from tsqr_factor
    B3 = bd.clone()
    assert torch.equal(outs[0][0].apply_qt_(B3), f.apply_qt_(bd.clone()))


def test_factor_solve_argument_errors(tl):
    A = dev(synth.gaussian(1000, 8, seed=1))
    b = dev(np.ones((1000, 1)))
    with pytest.raises(tl.TSQRError) as ei:
        tl.factor_solve(A, b, tl.opts(keep_q=False))
    assert ei.value.code == tl.ERR_STATE
    with pytest.raises(tl.TSQRError) as ei:
        tl.factor_solve(A, dev(np.ones((1000, 3))), tl.opts(lsq_max_rhs=2))
    assert ei.value.code == -8


def test_deterministic_and_r_only(tl):
    A = synth.gaussian(50000, 48, seed=9)
    Ad = dev(A)
    f1 = tl.factor(Ad, row_block=2000)
    f2 = tl.factor(Ad, row_block=2000)
    assert torch.equal(f1.R(), f2.R())
    assert torch.equal(f1.form_q(), f2.form_q())
    f3 = tl.factor(Ad, row_block=2000, keep_q=False)
    assert torch.equal(f3.R(), f1.R())
    with pytest.raises(tl.TSQRError) as ei:
        f3.form_q()
    assert ei.value.code == tl.ERR_STATE


def test_large_config_sampled(tl):
    """1,048,576 x 64 N(0,1), 4096-row domains, binary tree: R compared in
    full, Q compared on sampled rows plus the global identities."""
    A = synth.config_large()
    orc = oracle.TSQR(A, mb=4096)
    Ad = dev(A)
    f = tl.factor(Ad, row_block=4096)
    R = f.R()
    Ro = orc.R()
    assert rel(host(R), Ro) <= 1e-12
    Q = f.form_q()
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([rng.integers(0, A.shape[0], 2000),
                                     [0, 63, 64, 4095, 4096, A.shape[0] - 1]]))
    Qo = orc.form_q()
    assert rel(host(Q[torch.as_tensor(rows, device="cuda")]), Qo[rows]) <= 1e-12
    colwise(host(Q[torch.as_tensor(rows, device="cuda")]), Qo[rows], 1e-12,
            scale=np.linalg.norm(Qo[rows], axis=0))
    r_entrywise(host(R), Ro)
    # global identities in FP64 on the device (torch matmul only checks)
    G = Q.t() @ Q
    assert float(torch.linalg.norm(G - torch.eye(64, dtype=torch.float64, device="cuda"))) <= 1e-13
    E = Ad - Q @ R
    assert float(torch.linalg.norm(E) / torch.linalg.norm(Ad)) <= 1e-13
    # the benchmark's right-hand side (seed 1): x against the oracle's x,
    # through the separate solve and through the fused factor-solve call
    b = synth.config_large_rhs()
    Xo, reso, _ = orc.lsq(b)
    X, res, info = f.lsq(dev(b.reshape(-1, 1)))
    o = tl.opts(row_block=4096, lsq_max_rhs=1)
    _, X2, res2, info2 = tl.factor_solve(Ad, dev(b.reshape(-1, 1)), o)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and int(info2.item()) == 0
    kappa = np.linalg.cond(Ro)
    tan = reso[0] / np.linalg.norm(A @ Xo[:, 0])
    tol = max(1e-12, 10 * (kappa + kappa ** 2 * tan) * U)
    for Xg in (host(X), host(X2)):
        assert rel(Xg[:, 0], Xo[:, 0]) <= tol
        assert np.max(np.abs(Xg[:, 0] - Xo[:, 0])) <= tol * np.linalg.norm(Xo[:, 0])
    assert abs(host(res)[0] - reso[0]) <= 1e-11 * reso[0]
    assert torch.equal(X, X2)
