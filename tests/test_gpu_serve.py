"""GPU tests of the least-squares server (continuous batching, HBM-budget
admission, factor cache).

The key property: every request's result is the same alone (a fresh server
holding only that request) and in the mix (many requests admitted while
others run, sharing streams, with cached factors and evictions).  A request's
plan depends only on its own (m, n), so the two runs execute the same
kernels on the same data and must agree exactly; both must also meet the
accuracy bar against the FP64 oracle (x within max(1e-12, 10 kappa_LS u),
backward-error proxy eta <= 1e-12), including the requests at kappa = 1e6.
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


def host_cm(a):
    """Pinned, column-major float64 host tensor."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    t = torch.empty((a.shape[1], a.shape[0]), dtype=torch.float64, pin_memory=True)
    t.copy_(torch.as_tensor(np.ascontiguousarray(a.T)))
    return t.t()


def outputs(n, k):
    X = torch.zeros((k, n), dtype=torch.float64, pin_memory=True).t()
    res = torch.zeros(k, dtype=torch.float64, pin_memory=True)
    info = torch.full((1,), -7, dtype=torch.int32, pin_memory=True)
    return X, res, info


def eta(A, x, b):
    r = b - A @ x
    nA = np.linalg.norm(A)
    return float(np.linalg.norm(A.T @ r) / (nA * (nA * np.linalg.norm(x) + np.linalg.norm(b))))


@pytest.fixture(scope="module")
def stream_reqs():
    reqs = synth.serving_stream(28, seed=0, log2_lo=10, log2_hi=14, ill_frac=0.15)
    mats = {}
    for r in reqs:
        if r["matrix_id"] not in mats:
            mats[r["matrix_id"]] = synth.request_matrix(r["m"], r["n"], r["ill"], r["matrix_id"])
    rhs = {r["id"]: synth.request_rhs(r["m"], r["k"], r["rhs_seed"]) for r in reqs}
    return reqs, mats, rhs


def run(tl, reqs, mats, rhs, **kw):
    S = tl.Server(**kw)
    Ah = {mid: host_cm(A) for mid, A in mats.items()}
    out = {}
    tickets = {}
    for r in reqs:
        X, res, info = outputs(r["n"], r["k"])
        out[r["id"]] = (X, res, info)
        tickets[r["id"]] = S.submit(r["matrix_id"], Ah[r["matrix_id"]], host_cm(rhs[r["id"]]), X, res, info)
        S.progress()
    S.drain()
    st = S.stats()
    for r in reqs:
        assert S.status(tickets[r["id"]]) == 1, r
    S.close()
    return out, st


def test_server_mix_equals_alone_and_oracle(tl, stream_reqs):
    reqs, mats, rhs = stream_reqs
    print(f"case server mix of {len(reqs)} requests, budget 128 MiB", flush=True)
    mix, st = run(tl, reqs, mats, rhs, hbm_budget=128 << 20, streams=4, max_inflight=6)
    print(f"stats {st}", flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["bytes_peak"] <= 128 << 20
    assert st["cache_hits"] >= 1
    for r in reqs:
        alone, _ = run(tl, [r], {r["matrix_id"]: mats[r["matrix_id"]]}, rhs, hbm_budget=128 << 20,
                       streams=1, max_inflight=1, cache=False)
        Xm, rm, im = mix[r["id"]]
        Xa, ra, ia = alone[r["id"]]
        assert int(im[0]) == int(ia[0]) == 0
        assert torch.equal(Xm, Xa), f"request {r['id']} differs alone vs in the mix"
        assert torch.equal(rm, ra)
        A, B = mats[r["matrix_id"]], rhs[r["id"]]
        orc = oracle.TSQR(A, mb=max(r["n"], 4096))
        Xo, reso, _ = orc.lsq(B)
        kappa = np.linalg.cond(orc.R())
        X = Xm.numpy()
        for c in range(r["k"]):
            tan = reso[c] / max(np.linalg.norm(A @ Xo[:, c]), 1e-300)
            tol = max(1e-12, 10 * (kappa + kappa ** 2 * tan) * U)
            assert np.linalg.norm(X[:, c] - Xo[:, c]) <= tol * np.linalg.norm(Xo[:, c])
            assert eta(A, X[:, c], B[:, c]) <= 1e-12
            assert abs(rm[c].item() - reso[c]) <= 1e-10 * reso[c] + 1e-14 * np.linalg.norm(B[:, c])


def test_server_budget_forces_waits_and_evictions(tl, stream_reqs):
    reqs, mats, rhs = stream_reqs
    # just above the largest single request: at most a couple fit at once
    S = tl.Server(hbm_budget=40 << 20, streams=2, max_inflight=8)
    Ah = {mid: host_cm(A) for mid, A in mats.items()}
    keep = []
    for r in reqs:
        X, res, info = outputs(r["n"], r["k"])
        try:
            t = S.submit(r["matrix_id"], Ah[r["matrix_id"]], host_cm(rhs[r["id"]]), X, res, info)
        except tl.TSQRError as e:
            assert e.code == tl.ERR_WORKSPACE
            continue
        keep.append((t, r, X, info))
    S.drain()
    st = S.stats()
    S.close()
    assert st["bytes_peak"] <= 40 << 20
    assert st["evictions"] >= 1
    for t, r, X, info in keep:
        assert int(info[0]) == 0
        A, B = mats[r["matrix_id"]], rhs[r["id"]]
        assert eta(A, X.numpy()[:, 0], B[:, 0]) <= 1e-12


@pytest.mark.parametrize("route_kappa", [None, 0.0])
def test_server_mixed_precision(tl, route_kappa):
    """A mixed-precision server; by default the kappa = 1e6 request is routed
    to FP64 by its condition estimate (route_kappa 1e4), with routing off it
    is refined; every solution reaches eta <= 1e-12 either way."""
    reqs = [
        {"id": 0, "matrix_id": 0, "m": 6000, "n": 32, "k": 2, "ill": False, "rhs_seed": 1},
        {"id": 1, "matrix_id": 1, "m": 9000, "n": 128, "k": 1, "ill": True, "rhs_seed": 2},
        {"id": 2, "matrix_id": 0, "m": 6000, "n": 32, "k": 3, "ill": False, "rhs_seed": 3},
    ]
    mats = {0: synth.request_matrix(6000, 32, False, 0), 1: synth.request_matrix(9000, 128, True, 1)}
    rhs = {r["id"]: synth.request_rhs(r["m"], r["k"], r["rhs_seed"]) for r in reqs}
    print(f"case server mixed precision route_kappa={route_kappa}", flush=True)
    kw = {} if route_kappa is None else {"route_kappa": route_kappa}
    out, st = run(tl, reqs, mats, rhs, hbm_budget=256 << 20, prec=tl.MIXED, **kw)
    assert st["cache_hits"] == 1
    for r in reqs:
        X, res, info = out[r["id"]]
        assert int(info[0]) == 0
        A, B = mats[r["matrix_id"]], rhs[r["id"]]
        for c in range(r["k"]):
            assert eta(A, X.numpy()[:, c], B[:, c]) <= 1e-12


def test_server_rejects(tl):
    S = tl.Server(hbm_budget=8 << 20, streams=1)
    A = host_cm(np.ones((100000, 64)))
    B = host_cm(np.ones((100000, 1)))
    X, res, info = outputs(64, 1)
    with pytest.raises(tl.TSQRError) as e:
        S.submit(1, A, B, X, res, info)
    assert e.value.code == tl.ERR_WORKSPACE
    A2 = host_cm(np.random.default_rng(0).standard_normal((500, 8)))
    B2 = host_cm(np.ones((500, 1)))
    X2, r2, i2 = outputs(8, 1)
    S.submit(2, A2, B2, X2, r2, i2)
    A3 = host_cm(np.ones((600, 8)))
    with pytest.raises(tl.TSQRError) as e:
        S.submit(2, A3, host_cm(np.ones((600, 1))), *outputs(8, 1))
    assert e.value.code == -4
    S.drain()
    assert S.status(0) == 1
    S.close()


def _up(x):
    return (x + 255) // 256 * 256


def test_server_cache_hit_cannot_evict_its_own_entry(tl):
    """A repeat request whose cached factor is the only idle entry and splits
    the free memory so that its buffers fit nowhere: the entry it is about
    to use must not be evicted from under it.  The budget is computed so
    that exactly this happens: after the first request, the free space is
    [0, io_1) and [io_1 + entry, budget), both smaller than the second
    request's buffers.  The server must drop the idle entry and admit the
    request as a new matrix, with a correct result."""
    m, n = 50000, 4
    o = tl.opts(lsq_max_rhs=8)
    entry = _up(tl.workspace_bytes(m, n, o))
    io = lambda k, with_a: (_up(8 * m * k) + _up(8 * n * k) + _up(64) + _up(4)
                            + (_up(8 * m * n) if with_a else 0))
    budget = entry + io(8, True) + 4096
    assert budget - io(1, True) - entry < io(8, False) and io(1, True) < io(8, False)
    A = synth.request_matrix(m, n, False, 77)
    B1 = synth.request_rhs(m, 1, 1)
    B2 = synth.request_rhs(m, 8, 2)
    print(f"case cache hit under a tight budget ({budget} bytes)", flush=True)
    S = tl.Server(hbm_budget=budget, streams=1, max_inflight=2)
    Ah = host_cm(A)
    X1, r1, i1 = outputs(n, 1)
    S.submit(5, Ah, host_cm(B1), X1, r1, i1)
    S.drain()
    X2, r2, i2 = outputs(n, 8)
    S.submit(5, Ah, host_cm(B2), X2, r2, i2)
    S.drain()
    st = S.stats()
    S.close()
    assert st["completed"] == 2 and st["failed"] == 0
    assert st["bytes_peak"] <= budget
    assert st["evictions"] >= 1
    assert int(i1[0]) == 0 and int(i2[0]) == 0
    Xo, _, _ = oracle.TSQR(A, mb=4096).lsq(B2)
    assert rel_cols(X2.numpy(), Xo) <= 1e-12
    assert eta(A, X1.numpy()[:, 0], B1[:, 0]) <= 1e-12


def rel_cols(X, Xo):
    return max(float(np.linalg.norm(X[:, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c])) for c in range(Xo.shape[1]))


def test_server_mixed_solve_does_not_block(tl):
    """A mixed-precision solve synchronises once per refinement sweep; the
    server enqueues it from a worker thread, so a small request queued
    behind a long mixed request is admitted at once and retired as soon as
    it finishes, while the long one still refines."""
    big = {"m": 1 << 20, "n": 64, "ill": True}
    Ab = synth.request_matrix(big["m"], big["n"], True, 11)
    As = synth.request_matrix(5000, 16, False, 12)
    Bb = synth.request_rhs(big["m"], 2, 3)
    Bs = synth.request_rhs(5000, 1, 4)
    print("case mixed server: a long refinement does not hold the queue", flush=True)
    S = tl.Server(hbm_budget=8 << 30, streams=2, max_inflight=4, prec=tl.MIXED)
    Xb, rb, ib = outputs(big["n"], 2)
    Xs, rs, is_ = outputs(16, 1)
    tb = S.submit(1, host_cm(Ab), host_cm(Bb), Xb, rb, ib)
    ts = S.submit(2, host_cm(As), host_cm(Bs), Xs, rs, is_)
    while S.progress() > 0:
        pass
    sub_b, adm_b, done_b = S.times(tb)
    sub_s, adm_s, done_s = S.times(ts)
    S.close()
    print(f"big: admitted +{(adm_b - sub_b) * 1e3:.2f} ms, done +{(done_b - sub_b) * 1e3:.2f} ms; "
          f"small: admitted +{(adm_s - sub_s) * 1e3:.2f} ms, done +{(done_s - sub_s) * 1e3:.2f} ms", flush=True)
    assert int(ib[0]) == 0 and int(is_[0]) == 0
    assert adm_s - sub_s < 0.25 * (done_b - sub_b)
    assert done_s < done_b
    for c in range(2):
        assert eta(Ab, Xb.numpy()[:, c], Bb[:, c]) <= 1e-12
    assert eta(As, Xs.numpy()[:, 0], Bs[:, 0]) <= 1e-12


@pytest.mark.parametrize("bypass_ms", [0, -1])
def test_server_bypass_admission(tl, bypass_ms):
    """A request that does not fit beside a running one waits; a younger
    small request that fits is admitted past it within the bypass window
    (default), and not under strict FIFO (bypass_ms < 0)."""
    shapes = [(200000, 64), (300000, 64), (5000, 16)]
    mats = [synth.request_matrix(m, n, False, 20 + i) for i, (m, n) in enumerate(shapes)]
    rhs = [synth.request_rhs(m, 1, 30 + i) for i, (m, n) in enumerate(shapes)]
    o = tl.opts(lsq_max_rhs=8)
    need = [_up(tl.workspace_bytes(m, n, o)) + _up(8 * m) + _up(8 * n) + _up(64) + _up(4) + _up(8 * m * n)
            for m, n in shapes]
    budget = need[0] + need[2] + (need[1] - need[2]) // 2
    assert need[0] + need[1] > budget and need[1] <= budget
    print(f"case bypass_ms={bypass_ms}", flush=True)
    S = tl.Server(hbm_budget=budget, streams=2, max_inflight=4, cache=False, bypass_ms=bypass_ms)
    outs, tickets = [], []
    for i, (m, n) in enumerate(shapes):
        X, r, inf = outputs(n, 1)
        outs.append((X, r, inf))
        tickets.append(S.submit(i, host_cm(mats[i]), host_cm(rhs[i]), X, r, inf))
    S.progress()          # admits the first; the second does not fit beside it
    admitted = [S.times(t)[1] > 0 for t in tickets]
    S.drain()
    S.close()
    assert admitted[0] and not admitted[1]
    assert admitted[2] == (bypass_ms >= 0)
    for i in range(3):
        assert int(outs[i][2][0]) == 0
        assert eta(mats[i], outs[i][0].numpy()[:, 0], rhs[i][:, 0]) <= 1e-12


def test_server_large_requests_against_oracle(tl):
    """Requests at the top of the serving stream's range: n = 256 at
    m = 2^20 and a kappa = 1e6 request, in the mix with a small one, each
    compared with the FP64 oracle (E2 per right-hand side, eta)."""
    reqs = [
        {"id": 0, "matrix_id": 0, "m": 1 << 20, "n": 256, "k": 2, "ill": False, "rhs_seed": 7},
        {"id": 1, "matrix_id": 1, "m": 1 << 18, "n": 128, "k": 3, "ill": True, "rhs_seed": 8},
        {"id": 2, "matrix_id": 2, "m": 3000, "n": 16, "k": 1, "ill": False, "rhs_seed": 9},
    ]
    mats = {r["matrix_id"]: synth.request_matrix(r["m"], r["n"], r["ill"], r["matrix_id"]) for r in reqs}
    rhs = {r["id"]: synth.request_rhs(r["m"], r["k"], r["rhs_seed"]) for r in reqs}
    print("case server large requests (2^20 x 256, kappa 1e6 at 2^18 x 128)", flush=True)
    out, st = run(tl, reqs, mats, rhs, hbm_budget=12 << 30, streams=3, max_inflight=3)
    assert st["completed"] == 3 and st["failed"] == 0
    for r in reqs:
        X, res, info = out[r["id"]]
        assert int(info[0]) == 0
        A, B = mats[r["matrix_id"]], rhs[r["id"]]
        orc = oracle.TSQR(A, mb=4096)
        Xo, reso, _ = orc.lsq(B)
        kappa = np.linalg.cond(orc.R())
        Xh = X.numpy()
        for c in range(r["k"]):
            tan = reso[c] / max(np.linalg.norm(A @ Xo[:, c]), 1e-300)
            tol = max(1e-12, 10 * (kappa + kappa ** 2 * tan) * U)
            e2 = float(np.linalg.norm(Xh[:, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]))
            e1 = eta(A, Xh[:, c], B[:, c])
            print(f"request {r['id']} rhs {c}: kappa {kappa:.1e} E1 {e1:.2e} E2 {e2:.2e} (bound {tol:.1e})",
                  flush=True)
            assert e2 <= tol
            assert e1 <= 1e-12
