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


def test_server_mixed_precision(tl):
    reqs = [
        {"id": 0, "matrix_id": 0, "m": 6000, "n": 32, "k": 2, "ill": False, "rhs_seed": 1},
        {"id": 1, "matrix_id": 1, "m": 9000, "n": 128, "k": 1, "ill": True, "rhs_seed": 2},
        {"id": 2, "matrix_id": 0, "m": 6000, "n": 32, "k": 3, "ill": False, "rhs_seed": 3},
    ]
    mats = {0: synth.request_matrix(6000, 32, False, 0), 1: synth.request_matrix(9000, 128, True, 1)}
    rhs = {r["id"]: synth.request_rhs(r["m"], r["k"], r["rhs_seed"]) for r in reqs}
    print("case server mixed precision", flush=True)
    out, st = run(tl, reqs, mats, rhs, hbm_budget=256 << 20, prec=tl.MIXED)
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
