"""GPU parity of TSLU (tsqr_tslu): LU with tournament pivoting along the
TSQR partition and tree, against the oracle run on the same domains, stack
sizes (256 rows: a domain's first 256, then its b candidates on the next
256 - b) and schedule.

The pivot rows are compared exactly (they are integers decided by FP64
comparisons on both sides; the seeded Gaussian inputs leave no near-ties),
U and L within 1e-13 of their scale, info exactly; A = L U on the GPU's own
result.
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


def host(t):
    return t.detach().cpu().numpy()


def check_tslu(tl, A, o, tree):
    m, b = A.shape
    ipiv, L, U, info = tl.tslu(dev(A), o)
    torch.cuda.synchronize()
    ipiv, L, U, info = host(ipiv), host(L), host(U), int(info.item())
    parts = tl.partition(m, b, o)
    sched = tl.tree_schedule(len(parts), tree) if tree == tl.TREE_XCD else None
    ipo, Lo, Uo, info_o = oracle.tslu(A, parts, first=256, stage=256 - b, tree=tree, sched=sched)
    assert info == info_o
    assert ipiv.tolist() == ipo.tolist()
    su = np.maximum(np.abs(Uo).max(axis=0), 1e-300)
    assert np.all(np.abs(U - Uo) <= 1e-13 * su[None, :]), float(np.max(np.abs(U - Uo) / su[None, :]))
    assert np.all(np.tril(U, -1) == 0.0)
    assert np.max(np.abs(L - Lo)) <= 1e-12 * max(1.0, np.abs(Lo).max())
    L11 = L[ipiv]
    assert np.all(np.triu(L11, 1) == 0.0) and np.all(np.diag(L11) == 1.0)
    assert np.linalg.norm(A - L @ U) <= 1e-14 * np.sqrt(m) * np.linalg.norm(A)
    return ipiv, L, U, info


@pytest.mark.parametrize("m,b,mb,domains,tree", [
    (5000, 8, 1000, 0, 2),
    (20000, 16, 4096, 0, 4),
    (70001, 64, 4096, 0, 2),
    (100003, 33, 2048, 0, 0),
    (65536, 64, 4096, 0, 8),
    (300000, 64, 0, 256, 2),    # load-balanced domains
    (64, 64, 64, 0, 2),         # one stack of exactly b rows
    (1000, 1, 128, 0, 2),
    (4097, 50, 700, 0, 2),      # ragged domains and stages
])
def test_tslu_against_oracle(tl, m, b, mb, domains, tree):
    print(f"case tslu m={m} b={b} mb={mb} domains={domains} tree={tree}", flush=True)
    A = synth.gaussian(m, b, seed=m + b)
    o = tl.opts(domains=domains, tree=tree) if domains else tl.opts(row_block=mb, tree=tree)
    check_tslu(tl, A, o, tree)


def test_tslu_zero_column_info(tl):
    m, b = 9000, 12
    A = synth.gaussian(m, b, seed=2)
    A[:, 5] = 0.0
    print("case tslu zero column", flush=True)
    ipiv, L, U, info = check_tslu(tl, A, tl.opts(row_block=2000), 2)
    assert info == 6 and U[5, 5] == 0.0


def test_tslu_argument_errors(tl):
    with pytest.raises(ValueError):
        tl.tslu(dev(np.ones((100, 65))))     # b > 64
    with pytest.raises(ValueError):
        tl.tslu(dev(np.ones((4, 8))))        # m < b
