"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers and lays them out; it holds none of the
factorization's arithmetic.  Every generator uses NumPy's PCG64
(``numpy.random.default_rng(seed)``).  Draws fill a C-order (m, n) array which
is then stored column-major (Fortran order), the layout the library takes.

The paper's own workloads are dense FP64 tall-and-skinny matrices with M from
131,072 to 33,554,432 rows and N in {64, 128, 256, 512} (Sec. 5.1, 5.3-5.5);
their value distribution is not stated, so entries are iid N(0, 1) here.
"""
from __future__ import annotations

import numpy as np


def gaussian(m: int, n: int, seed: int = 0, rng=None) -> np.ndarray:
    """m x n iid N(0,1), column-major float64."""
    rng = np.random.default_rng(seed) if rng is None else rng
    return np.asfortranarray(rng.standard_normal((m, n)))


def config_small(seed: int = 0):
    """4096 x 16 N(0,1) matrix and one right-hand side b ~ N(0,1) of length
    4096, drawn in that order from one stream; 1024-row domains."""
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((4096, 16)))
    b = rng.standard_normal(4096)
    return A, b


def config_large(m: int = 1 << 20, n: int = 64, seed: int = 0) -> np.ndarray:
    """The single-matrix throughput workload: 1,048,576 x 64 N(0,1)."""
    return gaussian(m, n, seed)


def config_large_rhs(m: int = 1 << 20, seed: int = 1) -> np.ndarray:
    """The single-matrix workload's right-hand side: b ~ N(0,1), seed 1."""
    return np.random.default_rng(seed).standard_normal(m)


def log_spaced_spectrum(n: int, lo_exp: float = -6.0) -> np.ndarray:
    """s_i = 10^(lo_exp * i / (n-1)), i = 0..n-1 (1 down to 10^lo_exp)."""
    if n == 1:
        return np.ones(1)
    return 10.0 ** (lo_exp * np.arange(n) / (n - 1))


def config_conditioned(m: int, n: int, orthonormalize, seed: int = 0, lo_exp: float = -6.0):
    """A = U diag(s) V^T with s log-spaced from 1 to 10^lo_exp.

    Draw order from one stream: G1 (m x n), G2 (n x n), b (m), x_true (n).
    ``orthonormalize(G)`` must return the sign-normalised thin Q of G; the
    caller supplies it (the tests pass the oracle's, other callers a library
    QR), so no factorization arithmetic lives here.
    Returns (A, b, b_consistent, x_true, s).
    """
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((m, n))
    G2 = rng.standard_normal((n, n))
    b = rng.standard_normal(m)
    x_true = rng.standard_normal(n)
    U = orthonormalize(np.asfortranarray(G1))
    V = orthonormalize(np.asfortranarray(G2))
    s = log_spaced_spectrum(n, lo_exp)
    A = np.asfortranarray((U * s) @ V.T)
    bc = A @ x_true
    return A, b, bc, x_true, s


def batch_shapes(count: int = 512, seed: int = 0, m_lo: int = 1000, m_hi: int = 200000,
                 n_choices=(8, 16, 32, 64)):
    """Shapes of the batched workload: m_j ~ U[m_lo, m_hi], n_j from n_choices.
    Matrix j is run in mixed precision iff j is odd."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.choice(np.array(n_choices), size=count)
    return [(int(m), int(n)) for m, n in zip(ms, ns)]


def batch_matrices(shapes, seed: int = 1):
    """N(0,1) matrix and one RHS per shape, from one stream (seed + 0)."""
    rng = np.random.default_rng(seed)
    out = []
    for m, n in shapes:
        A = np.asfortranarray(rng.standard_normal((m, n)))
        b = rng.standard_normal(m)
        out.append((A, b))
    return out


def serving_stream(count: int, seed: int = 0, log2_lo: int = 10, log2_hi: int = 21,
                   n_choices=(16, 32, 64, 128, 256), k_max: int = 8,
                   ill_frac: float = 0.10, repeat_frac: float = 0.25):
    """Least-squares request stream.

    Each request: m = floor(2^U(log2_lo, log2_hi)), n from n_choices (m >= n
    enforced by raising m), k in 1..k_max, a flag for condition number 1e6,
    a matrix seed, and, for a share ``repeat_frac`` of requests, the id of an
    earlier request whose matrix it reuses with fresh right-hand sides.
    Inter-arrival gaps are returned as unit-rate exponentials; the caller
    scales them by 1/lambda.
    """
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        if i > 0 and rng.random() < repeat_frac:
            j = int(rng.integers(0, i))
            base = reqs[j]
            src = base["matrix_id"]
            m, n, ill = base["m"], base["n"], base["ill"]
        else:
            src = i
            m = int(np.floor(2.0 ** rng.uniform(log2_lo, log2_hi)))
            n = int(rng.choice(np.array(n_choices)))
            m = max(m, n)
            ill = bool(rng.random() < ill_frac)
        k = int(rng.integers(1, k_max + 1))
        reqs.append({"id": i, "matrix_id": src, "m": m, "n": n, "k": k, "ill": ill,
                     "gap": float(rng.exponential(1.0)), "rhs_seed": 100000 + i})
    return reqs


def request_matrix(m: int, n: int, ill: bool, matrix_id: int, lo_exp: float = -6.0):
    """Matrix of a serving request: N(0,1), or for ill-conditioned requests
    G diag(s) W / sqrt(m) with G N(0,1) (m x n), W a random signed
    permutation and s log-spaced from 1 to 10^lo_exp, so that cond(A) lies
    within cond(G) of 10^(-lo_exp)."""
    rng = np.random.default_rng(1000003 + matrix_id)
    G = rng.standard_normal((m, n))
    if not ill:
        return np.asfortranarray(G)
    s = log_spaced_spectrum(n, lo_exp)
    perm = rng.permutation(n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    A = (G * s)[:, perm] * sign
    return np.asfortranarray(A / np.sqrt(m))


def request_rhs(m: int, k: int, seed: int):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, k)))


def spd_gram(n: int, seed: int = 0, k: int = 0) -> np.ndarray:
    """Symmetric positive definite n x n Gram matrix A = G G^T / k of an
    n x k iid N(0,1) matrix G (k = 2n by default: eigenvalues in about
    [(1 - 1/sqrt 2)^2, (1 + 1/sqrt 2)^2], condition number about 34),
    column-major float64.  The Gram matrix of a block of vectors is what a
    Cholesky-based orthogonalisation factors."""
    k = 2 * n if k <= 0 else k
    G = np.random.default_rng(seed).standard_normal((n, k))
    A = (G @ G.T) / k
    A = 0.5 * (A + A.T)
    return np.asfortranarray(A)


def spd_gram_factor(n: int, seed: int = 0, k: int = 0) -> np.ndarray:
    """The G of spd_gram (n x k, C order), for callers that form G G^T / k
    on the device."""
    k = 2 * n if k <= 0 else k
    return np.random.default_rng(seed).standard_normal((n, k))

