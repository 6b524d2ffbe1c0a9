"""GPU parity of the Cholesky factorization (tsqr_cholesky) against the
oracle's column-by-column definition.

Tolerance: for an SPD A with condition number kappa the computed factor's
error is about n u kappa |L| entry by entry (the factorization is backward
stable, |E| <= gamma_{n+1} |L| |L^T|, and the forward error picks up
kappa); the Gram inputs here have kappa ~ 34, so |L - L_oracle| <= 4 n u 34
max|L| leaves a margin of about 4 over what both orders of summation can
differ by.  Exact checks: the info word, the untouched strict upper
triangle, and exact power-of-two scaling.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
KAPPA = 34.0


@pytest.fixture(scope="module")
def tl():
    import paper_0912_2572_amd as t
    t.lib()
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return t


def dev(x, ld=None):
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    ld = n if ld is None else ld
    buf = torch.full((x.shape[1], ld), float("nan"), dtype=torch.float64)
    buf[:, :n] = torch.as_tensor(x.T)
    return buf.cuda().t()[:n, :]


def run(tl, A, ld=None):
    n = A.shape[0]
    a = dev(A, ld)
    info = tl.cholesky(a)
    torch.cuda.synchronize()
    return a.cpu().numpy(), int(info.item())


def tol(n, L):
    return 4.0 * max(n, 1) * U * KAPPA * max(1.0, float(np.abs(L).max()))


@pytest.mark.parametrize("n,ld", [(1, 1), (5, 7), (63, 63), (64, 64), (65, 80), (100, 100), (255, 255),
                                  (256, 260), (257, 257), (300, 300), (520, 520), (777, 800), (1100, 1100)])
def test_cholesky_matches_oracle(tl, n, ld):
    A = synth.spd_gram(n, seed=500 + n)
    # the strict upper triangle carries a sentinel: never read, never written
    Au = A.copy(order="F")
    Au[np.triu_indices(n, 1)] = -7.25
    G, info = run(tl, Au, ld)
    Lo, info_o = oracle.cholesky(A)
    assert info == 0 and info_o == 0
    L = np.tril(G)
    assert np.all(G[np.triu_indices(n, 1)] == -7.25)
    err = float(np.max(np.abs(L - Lo)))
    assert err <= tol(n, Lo), err
    assert np.all(np.diag(L) > 0)


def test_cholesky_power_of_two_scaling_is_exact(tl):
    n = 333
    A = synth.spd_gram(n, seed=17)
    e = np.random.default_rng(18).integers(-40, 41, n)
    D = np.ldexp(1.0, e)
    G0, i0 = run(tl, A)
    G1, i1 = run(tl, D[:, None] * A * D[None, :])
    assert i0 == 0 and i1 == 0
    assert np.array_equal(np.tril(G1), D[:, None] * np.tril(G0))


@pytest.mark.parametrize("n,j", [(300, 0), (300, 150), (300, 255), (300, 256), (300, 299), (70, 66)])
def test_cholesky_info_on_indefinite(tl, n, j):
    A = synth.spd_gram(n, seed=40 + j)
    A[j, j] = -1.0
    G, info = run(tl, A)
    Lo, info_o = oracle.cholesky(A)
    assert info_o == j + 1 and info == j + 1
    done = (j // 64) * 64        # the columns before the failing 64-column panel are final
    if done:
        err = float(np.max(np.abs(np.tril(G)[:, :done] - Lo[:, :done])))
        assert err <= tol(n, Lo[:, :done]), err


def test_cholesky_nan_and_zero_size(tl):
    A = synth.spd_gram(50, seed=3)
    A[0, 0] = np.nan
    assert run(tl, A)[1] == 1
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    a = torch.empty((0, 0), dtype=torch.float64, device="cuda")
    tl.cholesky(a, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0


def test_cholesky_after_failure_next_call_succeeds(tl):
    # the info word is cleared by every call, so a failed call does not
    # stop the next one
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    A = synth.spd_gram(200, seed=5)
    B = A.copy(order="F")
    B[10, 10] = -3.0
    b = dev(B)
    tl.cholesky(b, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 11
    a = dev(A)
    tl.cholesky(a, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Lo, _ = oracle.cholesky(A)
    assert float(np.max(np.abs(np.tril(a.cpu().numpy()) - Lo))) <= tol(200, Lo)


def test_cholesky_large_leading_block_and_backward_error(tl):
    # n = 8192 (the benchmark size, 128 panels, 31 block columns): the factor
    # of a leading principal block is the leading block of L, so the oracle
    # checks L[:1600, :1600]; every sampled entry of L L^T must equal A to
    # the backward-error bound.
    n, lead = 8192, 1600
    G = synth.spd_gram_factor(n, seed=81)
    g = torch.as_tensor(G).cuda()
    a = (g @ g.t()) / (2 * n)
    a = 0.5 * (a + a.t())
    A_lead = a[:lead, :lead].cpu().numpy()
    rng = np.random.default_rng(82)
    ii = rng.integers(0, n, 4000)
    jj = rng.integers(0, n, 4000)
    ii, jj = np.maximum(ii, jj), np.minimum(ii, jj)
    A_s = a[ii, jj].cpu().numpy()
    del g
    a = a.t().contiguous().t()   # column-major (symmetric, so the same values)
    info = tl.cholesky(a)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    L = torch.tril(a)
    Lo, info_o = oracle.cholesky(A_lead)
    assert info_o == 0
    Lg = L[:lead, :lead].cpu().numpy()
    err = float(np.max(np.abs(Lg - Lo)))
    assert err <= tol(lead, Lo), err
    li = L[torch.as_tensor(ii).cuda()]
    lj = L[torch.as_tensor(jj).cuda()]
    rec = (li * lj).sum(dim=1).cpu().numpy()
    bound = (n + 1) * U * (li.abs() * lj.abs()).sum(dim=1).cpu().numpy()
    assert np.all(np.abs(rec - A_s) <= 4.0 * bound), float(np.max(np.abs(rec - A_s) / bound))


def test_cholesky_on_a_side_stream_is_deterministic(tl):
    # the bulk of each trailing update runs on the library's second stream
    # beside the next panels; every call on a caller's stream must still see
    # the whole factorization done, and give the same bits each time
    n = 2000
    A = synth.spd_gram(n, seed=77)
    side = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(side):
        for _ in range(3):
            a = dev(A)
            side.wait_stream(torch.cuda.default_stream())
            info = tl.cholesky(a, stream=side)
            outs.append((a, info))
    side.synchronize()
    G = [o[0].cpu().numpy() for o in outs]
    assert all(int(o[1].item()) == 0 for o in outs)
    assert np.array_equal(G[0], G[1]) and np.array_equal(G[0], G[2])
    Lo, _ = oracle.cholesky(A)
    assert float(np.max(np.abs(np.tril(G[0]) - Lo))) <= tol(n, Lo)
