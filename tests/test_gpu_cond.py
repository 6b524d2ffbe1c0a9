"""GPU parity of the condition estimate of R (tsqr_cond_estimate) and of
the mixed-precision routing it drives (opts.route_kappa): an ill-conditioned
mixed solve is refactored and solved in FP64.

The estimate is compared with the oracle's estimate on the oracle's own R
(the same Hager-Higham steps; R differs from the GPU's by rounding, which
the solves amplify by up to kappa, hence a tolerance of 1e-10 + 1e-11 kappa
relative), and checked to be a lower bound of the exact kappa_1 within a
factor of 3.  A routed solve must equal the FP64 factor + solve bitwise (it
is that computation on the same workspace layout), a solve that is not
routed must equal the one with routing off bitwise.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import paper_0912_2572_amd as t
    t.lib()
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return t


def dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64)).t().contiguous().t().cuda()


def host(t):
    return t.detach().cpu().numpy()


def orth(G):
    return oracle.TSQR(G, mb=max(G.shape[1], 4096)).form_q()


def graded(m, n, decades, seed):
    A, _, _, _, _ = synth.config_conditioned(m, n, orth, seed=seed, lo_exp=-decades)
    return A


@pytest.mark.parametrize("m,n,decades,mb,prec", [
    (5000, 1, 0, 1000, "f64"),
    (20000, 13, 2, 4096, "f64"),
    (65536, 64, 6, 4096, "f64"),
    (65536, 64, 4, 4096, "mixed"),     # one panel: the mixed R is FP64-exact
    (30000, 100, 4, 2048, "f64"),     # two panels
    (20000, 256, 3, 4096, "f64"),     # four panels, 4 entries per lane
])
def test_cond_estimate_against_oracle(tl, m, n, decades, mb, prec):
    print(f"case cond m={m} n={n} kappa=1e{decades} mb={mb} {prec}", flush=True)
    A = graded(m, n, decades, seed=m + n)
    f = tl.factor(dev(A), row_block=mb, prec=tl.MIXED if prec == "mixed" else tl.F64)
    est = float(host(f.cond_estimate())[0])
    Ro = oracle.TSQR(A, mb=mb).R()
    est_o, ex = oracle.cond1_est(Ro), oracle.cond1(Ro)
    tol = 1e-10 + 1e-11 * ex
    print(f"  estimate {est:.6e}, oracle estimate {est_o:.6e}, kappa_1 {ex:.6e}", flush=True)
    assert abs(est - est_o) <= tol * est_o
    assert est <= ex * (1 + tol)
    assert est >= ex / 3


def test_cond_estimate_zero_diagonal_is_inf(tl):
    A = synth.gaussian(4000, 12, seed=5)
    A[:, 7] = 0.0
    f = tl.factor(dev(A), row_block=1000)
    assert math.isinf(float(host(f.cond_estimate())[0]))


def test_route_ill_conditioned_mixed_solve_to_f64(tl):
    m, n, mb = 65536, 128, 4096
    print(f"case route m={m} n={n} kappa=1e6", flush=True)
    A = graded(m, n, 6, seed=0)
    b = np.random.default_rng(1).standard_normal((m, 2))
    Ad, bd = dev(A), dev(b)
    f = tl.factor(Ad, row_block=mb, prec=tl.MIXED, route_kappa=1e4)
    X, res, info = f.lsq(bd, A=Ad)
    Q = f.form_q()
    g = tl.factor(Ad, row_block=mb)
    X64, res64, info64 = g.lsq(bd)
    Q64 = g.form_q()
    torch.cuda.synchronize()
    prec, kap = f.route_info()
    print(f"  routed: prec {prec}, estimate {kap:.3e}", flush=True)
    assert prec == tl.F64 and kap > 1e4
    assert f.last_refine_iters() == 0
    assert int(info.item()) == int(info64.item()) == 0
    assert torch.equal(X, X64) and torch.equal(res, res64) and torch.equal(Q, Q64)
    assert torch.equal(f.R(), g.R())
    # the estimate that decided it came from the mixed factor's R, which for
    # two panels carries the FP32 trailing update's error (kappa_1 ~ 8e6 is
    # then known to a few digits): within a factor of 2 of the oracle's
    est_o = oracle.cond1_est(oracle.TSQR(A, mb=mb).R())
    print(f"  oracle estimate {est_o:.3e}", flush=True)
    assert est_o / 2 <= kap <= 2 * est_o


def test_well_conditioned_mixed_solve_is_not_routed(tl):
    m, n, mb = 40000, 48, 4096
    print(f"case no route m={m} n={n}", flush=True)
    A = synth.gaussian(m, n, seed=8)
    b = np.random.default_rng(9).standard_normal((m, 1))
    Ad, bd = dev(A), dev(b)
    f = tl.factor(Ad, row_block=mb, prec=tl.MIXED, route_kappa=1e4)
    X, res, info = f.lsq(bd, A=Ad)
    g = tl.factor(Ad, row_block=mb, prec=tl.MIXED)
    Xg, resg, infog = g.lsq(bd, A=Ad)
    torch.cuda.synchronize()
    prec, kap = f.route_info()
    assert prec == tl.MIXED and 1.0 <= kap <= 1e4
    assert g.route_info() == (tl.MIXED, 0.0)
    assert f.last_refine_iters() == g.last_refine_iters() >= 2
    assert torch.equal(X, Xg) and torch.equal(res, resg)
    # a second solve on the routed-or-not handle does not estimate again
    X2, _, _ = f.lsq(bd, A=Ad)
    torch.cuda.synchronize()
    assert torch.equal(X2, X)
