"""GPU parity of the batched path (tsqr_batch_*, tsqr_autotune).

A batch of independent matrices with uneven m and n (n in {8, 16, 32, 64}),
half FP64 and half mixed (odd index), one b ~ N(0,1) each, is factored and
solved in one run (captured HIP graph).  Every matrix is checked against the
FP64 oracle: R within 1e-12 after sign normalisation (with n <= 64 even the
mixed matrices have FP64 leaves and tree), x within max(1e-12, 10 kappa_LS u)
and the backward-error proxy eta <= 1e-12.  Graph replays, plain launches
and single-matrix calls with the same plan must give the same results.
"""
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


def eta(A, x, b):
    r = b - A @ x
    nA = np.linalg.norm(A)
    return float(np.linalg.norm(A.T @ r) / (nA * (nA * np.linalg.norm(x) + np.linalg.norm(b))))


@pytest.fixture(scope="module")
def small_batch():
    shapes = synth.batch_shapes(24, seed=0, m_lo=1000, m_hi=30000)
    return shapes, with_prec(synth.batch_matrices(shapes, seed=1))


def with_prec(pairs):
    # matrix j runs in mixed precision iff j is odd
    return [(A, b, j % 2) for j, (A, b) in enumerate(pairs)]


def make(tl, shapes, mats, **kw):
    As = [dev(A) for A, b, prec in mats]
    bs = [dev(b) for A, b, prec in mats]
    precs = [prec for A, b, prec in mats]
    return tl.Batch(As, bs, precs, **kw)


def check_against_oracle(tl, B, mats, mb_of):
    for i, (A, b, prec) in enumerate(mats):
        m, n = A.shape
        mb, tree, P = B.plan(i)
        assert mb == mb_of(i)
        orc = oracle.TSQR(A, mb=mb, tree=tree)
        Ro = orc.R()
        R = host(B.R(i))
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
        assert rel(R, Ro) <= 1e-12, f"matrix {i} ({m}x{n}, prec {prec})"
        assert int(B.info(i).item()) == 0
        x = host(B.x(i))
        Xo, reso, _ = orc.lsq(b)
        kappa = np.linalg.cond(Ro)
        tan = reso[0] / max(np.linalg.norm(A @ Xo[:, 0]), 1e-300)
        tol = max(1e-12, 10 * (kappa + kappa ** 2 * tan) * U)
        assert rel(x, Xo[:, 0]) <= tol, f"matrix {i}"
        assert eta(A, x, b) <= 1e-12, f"matrix {i}"
        r = np.linalg.norm(b - A @ x)
        assert abs(host(B.resid(i))[0] - r) <= 1e-10 * r


def test_batch_graph_matches_oracle(tl, small_batch):
    shapes, mats = small_batch
    print(f"case batch count={len(mats)} default plan, graph", flush=True)
    B = make(tl, shapes, mats)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B.run(use_graph=True, stream=stream)
    stream.synchronize()
    check_against_oracle(tl, B, mats, lambda i: max(4096, mats[i][0].shape[1]))


def test_batch_replays_and_plain_launches_agree(tl, small_batch):
    shapes, mats = small_batch
    print("case batch replay x3 vs plain launches", flush=True)
    B = make(tl, shapes, mats)
    B.run(use_graph=False)
    torch.cuda.synchronize()
    ref = [(host(B.R(i)).copy(), host(B.x(i)).copy()) for i in range(len(mats))]
    stream = torch.cuda.Stream()
    for rep in range(3):
        # the program's own eager work between replays
        for i in range(len(mats)):
            B.x(i).fill_(-1.0)
            B.R(i).fill_(0.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            B.run(use_graph=True, stream=stream)
        stream.synchronize()
        for i in range(len(mats)):
            assert np.array_equal(host(B.R(i)), ref[i][0]), f"replay {rep} matrix {i}"
            assert np.array_equal(host(B.x(i)), ref[i][1]), f"replay {rep} matrix {i}"


def test_batch_equals_single_calls(tl, small_batch):
    """Each matrix's R equals (bitwise) a single tsqr_factor with the same
    plan: the batched factor runs the same per-domain and per-chain code.
    An FP64 matrix's x equals the single call's bitwise too (the batched
    apply passes run the single-matrix bodies); a mixed matrix's refinement
    runs a fixed, device-gated sweep schedule, so its x agrees to rounding."""
    shapes, mats = small_batch
    print("case batch vs single calls", flush=True)
    B = make(tl, shapes, mats)
    B.run(use_graph=False)
    torch.cuda.synchronize()
    for i, (A, b, prec) in enumerate(mats[:10]):
        mb, tree, P = B.plan(i)
        f = tl.factor(dev(A), row_block=mb, tree=tree, prec=prec, lsq_max_rhs=1)
        assert np.array_equal(host(f.R()), host(B.R(i))), f"matrix {i}"
        X, res, info = f.lsq(dev(b.reshape(-1, 1)), A=dev(A))
        torch.cuda.synchronize()
        if prec == tl.F64:
            assert np.array_equal(host(X)[:, 0], host(B.x(i))), f"matrix {i}"
        else:
            assert rel(host(X)[:, 0], host(B.x(i))) <= 1e-13


def test_batch_tuned_plans(tl, small_batch):
    """A tuning table sets each class's plan; a matrix's plan depends only on
    (m, n, precision), not on the rest of the batch."""
    shapes, mats = small_batch
    tune = [{"n_max": 8, "prec": 0, "row_block": 1024, "tree": 4},
            {"n_max": 16, "prec": 0, "row_block": 2048, "tree": 0},
            {"n_max": 64, "prec": 0, "row_block": 512, "tree": 2},
            {"n_max": 64, "prec": 1, "row_block": 8192, "tree": 4}]
    print("case batch with a tuning table", flush=True)
    B = make(tl, shapes, mats, tune=tune)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B.run(use_graph=True, stream=stream)
    stream.synchronize()

    def mb_of(i):
        n, prec = mats[i][0].shape[1], mats[i][2]
        if prec == 1:
            return 8192
        return 1024 if n <= 8 else (2048 if n <= 16 else 512)
    check_against_oracle(tl, B, mats, mb_of)
    # the same matrices in another composition get the same plans and results
    sub = mats[::3]
    B2 = make(tl, None, sub, tune=tune)
    B2.run(use_graph=False)
    torch.cuda.synchronize()
    for j, i in enumerate(range(0, len(mats), 3)):
        assert B2.plan(j) == B.plan(i)
        assert np.array_equal(host(B2.R(j)), host(B.R(i)))
        assert np.array_equal(host(B2.x(j)), host(B.x(i)))


def test_autotune_small(tl):
    shapes = synth.batch_shapes(8, seed=3, m_lo=2000, m_hi=8000)
    mats = with_prec(synth.batch_matrices(shapes, seed=4))
    As = [dev(A) for A, b, p in mats]
    bs = [dev(b) for A, b, p in mats]
    precs = [p for A, b, p in mats]
    print("case autotune 8 matrices", flush=True)
    table = tl.autotune(As, bs, precs, reps=1)
    assert len(table) >= 1
    for e in table:
        assert e["row_block"] in (512, 1024, 2048, 4096, 8192)
        assert e["tree"] in (0, 2, 4)
        assert e["n_max"] in (8, 16, 32, 64) and e["prec"] in (0, 1)
    B = tl.Batch(As, bs, precs, tune=table)
    B.run(use_graph=False)
    torch.cuda.synchronize()
    for i, (A, b, prec) in enumerate(mats):
        assert int(B.info(i).item()) == 0
        assert eta(A, host(B.x(i)), b) <= 1e-12


def test_batch_zero_column(tl):
    rng = np.random.default_rng(9)
    A0 = rng.standard_normal((3000, 8))
    A0[:, 2] = 0.0
    A1 = rng.standard_normal((5000, 16))
    mats = [(A0, rng.standard_normal(3000), 0), (A0.copy(), rng.standard_normal(3000), 1),
            (A1, rng.standard_normal(5000), 1)]
    B = make(tl, None, mats)
    for i in range(3):
        B.x(i).fill_(7.0)
    B.run(use_graph=False)
    torch.cuda.synchronize()
    assert int(B.info(0).item()) == 3 and int(B.info(1).item()) == 3
    assert torch.all(B.x(0) == 7.0) and torch.all(B.x(1) == 7.0)
    assert int(B.info(2).item()) == 0
    assert eta(A1, host(B.x(2)), mats[2][1]) <= 1e-12


def test_batch_full_config_sampled(tl):
    """The full 512-matrix workload in the configuration the benchmark times
    (autotuned table, captured graph), checked against the oracle on a sample
    of matrices (the oracle factors them one by one)."""
    shapes = synth.batch_shapes(512, seed=0)
    precs = [j % 2 for j in range(len(shapes))]
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    As, bs = [], []
    for m, n in shapes:
        As.append(torch.randn((n, m), generator=g, device="cuda", dtype=torch.float64).t())
        bs.append(torch.randn(m, generator=g, device="cuda", dtype=torch.float64))
    print("case batch 512 matrices, autotuned, graph", flush=True)
    table = tl.autotune(As[::3], bs[::3], precs[::3], reps=1)
    B = tl.Batch(As, bs, precs, tune=table, refine_sweeps=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B.run(use_graph=True, stream=stream)
    stream.synchronize()
    for i in list(range(0, 512, 37)) + [511]:
        A, b = host(As[i]), host(bs[i])
        mb, tree, P = B.plan(i)
        orc = oracle.TSQR(A, mb=mb, tree=tree)
        Ro = orc.R()
        assert rel(host(B.R(i)), Ro) <= 1e-12, f"matrix {i}"
        Xo, reso, _ = orc.lsq(b)
        x = host(B.x(i))
        assert int(B.info(i).item()) == 0
        assert rel(x, Xo[:, 0]) <= 1e-12, f"matrix {i}"
        assert eta(A, x, b) <= 1e-12, f"matrix {i}"
