"""GPU parity of block orthogonalisation (tsqr_block_orth), the step that
block-iterative methods repeat with TSQR as the stable orthogonalisation of
each new block (the paper's Scope section and Sec. 6).

Against the FP64 oracle (two NumPy Gram-Schmidt passes and the oracle's
TSQR), column by column: Q (unique once diag(R) >= 0) within 1e-12, H and R
within 1e-12 of their column norms; and the identities W = V H + Q R and
[V Q]^T [V Q] = I within 1e-13 on the GPU's own results.  A block Krylov
loop (a diagonal operator applied to the last block, eight blocks) is
compared with the same loop run by the oracle.
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
    t = torch.as_tensor(np.asarray(x, dtype=np.float64))
    return t.t().contiguous().t().cuda()


def host(t):
    return t.detach().cpu().numpy()


def colwise(a, b, tol, scale):
    for j in range(b.shape[1]):
        err = np.linalg.norm(a[:, j] - b[:, j])
        assert err <= tol * scale[j], f"column {j}: {err:.3e} > {tol:.1e} * {scale[j]:.3e}"


@pytest.mark.parametrize("m,nv,b,mb", [
    (5000, 0, 8, 1000),        # first block: plain TSQR
    (4096, 16, 16, 1024),
    (20000, 24, 8, 4096),
    (30001, 40, 13, 2048),     # ragged rows, b not a multiple of 16
    (65536, 100, 33, 4096),    # nv not a multiple of 16 or 64
    (100003, 257, 64, 4096),   # several 64-column slices of V, the widest block
])
def test_block_orth_against_oracle(tl, m, nv, b, mb):
    print(f"case block_orth m={m} nv={nv} b={b} mb={mb}", flush=True)
    rng = np.random.default_rng(m + nv + b)
    V = np.asfortranarray(np.linalg.qr(rng.standard_normal((m, nv)))[0]) if nv else None
    W = synth.gaussian(m, b, seed=nv + b)
    Qo, Ho, Ro = oracle.block_orth(V, W, mb)
    Vd = dev(V) if nv else None
    Wd = dev(W)
    Q, H, R = tl.block_orth(Vd, Wd, tl.opts(row_block=mb))
    torch.cuda.synchronize()
    Q, R = host(Q), host(R)
    wn = np.linalg.norm(W, axis=0)
    colwise(Q, Qo, 1e-12, np.ones(b))
    colwise(R, Ro, 1e-12, wn)
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
    B = Q
    recon = Q @ R
    if nv:
        H = host(H)
        colwise(H, Ho, 1e-12, wn)
        B = np.hstack([V, Q])
        recon = V @ H + recon
    assert np.linalg.norm(B.T @ B - np.eye(B.shape[1])) <= 1e-13
    assert np.linalg.norm(recon - W) <= 1e-13 * np.linalg.norm(W)


def test_block_krylov_loop_against_oracle(tl):
    """Eight blocks of a block Krylov basis for a diagonal operator D: the
    next block is D Q_j, orthogonalised against all previous blocks; the
    GPU basis matches the oracle's loop and stays orthonormal."""
    m, b, nblocks = 50000, 16, 8
    d = np.linspace(1.0, 2.0, m)
    rng = np.random.default_rng(11)
    W0 = rng.standard_normal((m, b))
    print("case block Krylov loop 50000 x (8 x 16)", flush=True)
    # oracle loop
    Vo = None
    for j in range(nblocks):
        Wj = W0 if j == 0 else d[:, None] * Vo[:, -b:]
        Q, H, R = oracle.block_orth(Vo, Wj, 4096)
        Vo = Q if Vo is None else np.hstack([Vo, Q])
    # GPU loop on one basis buffer
    Vg = tl.empty_colmajor(m, nblocks * b, device="cuda")
    dd = torch.as_tensor(d, device="cuda")
    o = tl.opts(row_block=4096)
    for j in range(nblocks):
        Wj = Vg[:, j * b:(j + 1) * b]
        if j == 0:
            Wj.copy_(dev(W0))
            tl.block_orth(None, Wj, o)
        else:
            Wj.copy_(dd[:, None] * Vg[:, (j - 1) * b:j * b])
            tl.block_orth(Vg[:, :j * b], Wj, o)
    torch.cuda.synchronize()
    Vh = host(Vg)
    assert np.linalg.norm(Vh.T @ Vh - np.eye(nblocks * b)) <= 1e-12
    # the bases agree column by column (errors grow mildly over the blocks)
    for c in range(nblocks * b):
        assert np.linalg.norm(Vh[:, c] - Vo[:, c]) <= 1e-10, c


def test_block_orth_argument_errors(tl):
    import ctypes
    L = tl.lib()
    o = tl.opts()
    W = dev(np.ones((100, 8)))
    V = dev(np.eye(100)[:, :95])
    work = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    R = dev(np.zeros((8, 8)))
    H = dev(np.zeros((95, 8)))
    args = lambda nv, b, ldr: (100, nv, ctypes.c_void_p(V.data_ptr()), 100, b, ctypes.c_void_p(W.data_ptr()), 100,
                               ctypes.c_void_p(H.data_ptr()), 95, ctypes.c_void_p(R.data_ptr()), ldr,
                               ctypes.byref(o), ctypes.c_void_p(work.data_ptr()), work.numel(), None)
    assert L.tsqr_block_orth(*args(95, 8, 8)) == -2      # nv + b > m
    assert L.tsqr_block_orth(*args(10, 65, 65)) == -5    # b > 64
    assert L.tsqr_block_orth(*args(10, 8, 7)) == -11     # ldr < b
    assert L.tsqr_block_orth_workspace_bytes(100, 95, 8, ctypes.byref(o)) == 0
    with pytest.raises(ValueError):
        tl.block_orth(None, dev(np.ones((100, 65))))
