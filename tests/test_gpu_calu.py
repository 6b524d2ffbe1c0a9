"""GPU parity of CALU (tsqr_calu): LU with tournament-pivoted 64-column
panels, against the oracle run with the same row block and tree.

The interchanges are compared exactly: each pivot choice is an FP64
comparison on both sides and the seeded Gaussian inputs leave no near-ties,
so a rounding-level difference in the trailing matrix does not flip one.
The packed L\\U is compared to 1e-11 of its largest entry (the two sides
sum the trailing updates in different orders; Gaussian matrices of these
sizes have condition numbers up to ~1e4 and small pivot growth, so the
factors agree to ~1e-13); the GPU's own P A = L U is checked too.
"""
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


def parts(LU, ipiv):
    m, n = LU.shape
    L = np.tril(LU, -1)[:, :n] + np.eye(m, n)
    U = np.triu(LU[:n, :])
    perm = np.arange(m)
    for i, p in enumerate(ipiv):
        perm[[i, p]] = perm[[p, i]]
    return L, U, perm


def run(tl, A, o):
    a = dev(A)
    ipiv, info = tl.calu(a, o)
    torch.cuda.synchronize()
    return a.cpu().numpy(), ipiv.cpu().numpy(), int(info.item())


TREES = {"binary": 2, "quad": 4, "flat": 0}


@pytest.mark.parametrize("m,n,mb,tree", [
    (5, 5, 4096, "binary"), (100, 100, 4096, "binary"), (256, 130, 4096, "binary"), (90, 1, 4096, "binary"),
    (3000, 200, 512, "binary"), (2500, 130, 600, "quad"), (1500, 64, 256, "flat"), (800, 800, 300, "binary"),
    (4100, 65, 1024, "binary"), (2048, 1024, 256, "binary")])
def test_calu_matches_oracle(tl, m, n, mb, tree):
    A = synth.gaussian(m, n, seed=900 + m + n)
    o = tl.opts(row_block=mb, tree=TREES[tree])
    LU, ipiv, info = run(tl, A, o)
    LUo, ipo, info_o = oracle.calu(A, mb=mb, tree=TREES[tree])
    assert info == info_o == 0
    assert ipiv.tolist() == ipo.tolist()
    err = float(np.max(np.abs(LU - LUo)))
    assert err <= 1e-11 * max(1.0, float(np.abs(LUo).max())), err
    L, U, perm = parts(LU, ipiv)
    assert np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A) <= 1e-14 * np.sqrt(n)


def test_calu_zero_column_sets_info(tl):
    A = synth.gaussian(1200, 150, seed=31)
    A[:, 70] = 0.0
    o = tl.opts(row_block=400)
    LU, ipiv, info = run(tl, A, o)
    LUo, ipo, info_o = oracle.calu(A, mb=400)
    assert info == info_o == 71
    assert ipiv.tolist() == ipo.tolist()
    assert float(np.max(np.abs(LU - LUo))) <= 1e-11 * float(np.abs(LUo).max())


def test_calu_balanced_and_xcd_tree_reconstruct(tl):
    # partitions and trees the oracle does not take as options: the GPU's
    # own P A = L U, unit-bounded growth and a valid interchange sequence
    A = synth.gaussian(6000, 300, seed=41)
    for o in (tl.opts(domains=-1), tl.opts(row_block=700, tree=tl.TREE_XCD)):
        LU, ipiv, info = run(tl, A, o)
        assert info == 0
        assert np.all(ipiv >= np.arange(300)) and np.all(ipiv < 6000)
        L, U, perm = parts(LU, ipiv)
        assert np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A) <= 1e-14 * np.sqrt(300)
        assert np.abs(L).max() <= 16.0
