"""FP64 CPU oracle for TSQR -- test infrastructure only.

The oracle is the plain, slow reference that the GPU library is checked
against.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product package never does.

The arithmetic lives in ``tsqr_oracle.c`` (plain loops, IEEE double); this
module only builds it with gcc and marshals NumPy arrays through ctypes.
Every function cites the passage of Agullo et al. (arXiv 0912.2572) that it
follows; see the C file for the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsqr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

TREE_FLAT = 0
TREE_BINARY = 2
TREE_QUAD = 4
XCDS = 8          # clusters of the hierarchical GPU tree: domain d on XCD d mod 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=gnu11", "-fno-fast-math", "-ffp-contract=off",
             "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm", "-lquadmath"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, dp, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
        ip = ctypes.POINTER(ctypes.c_int64)
        L.or_larfg.argtypes = [i64, dp, dp, i64, dp]
        L.or_geqrt.argtypes = [i64, i64, dp, i64, dp, dp, i64]
        L.or_tpqrt.argtypes = [i64, dp, i64, dp, i64, dp, dp, i64]
        L.or_partition.argtypes = [i64, i64, i64, ip, ip]
        L.or_partition.restype = i64
        L.or_schedule.argtypes = [i64, ctypes.c_int, ip, ip]
        L.or_schedule.restype = i64
        L.or_factor.argtypes = [i64, i64, dp, i64, i64, ctypes.c_int, ctypes.c_int]
        L.or_factor.restype = vp
        L.or_factor_sched.argtypes = [i64, i64, dp, i64, i64, i64, ip, ip, ctypes.c_int]
        L.or_factor_sched.restype = vp
        L.or_partition_weighted.argtypes = [i64, i64, i64, i64, ip, ip, ip]
        L.or_partition_weighted.restype = i64
        L.or_factor_parts.argtypes = [i64, i64, dp, i64, i64, ip, ip, i64, ip, ip, ctypes.c_int]
        L.or_factor_parts.restype = vp
        L.or_free.argtypes = [vp]
        L.or_num_domains.argtypes = [vp]
        L.or_num_domains.restype = i64
        L.or_get_r.argtypes = [vp, dp, i64]
        L.or_get_leaf.argtypes = [vp, dp, dp, dp]
        L.or_apply_qt.argtypes = [vp, i64, dp, i64]
        L.or_form_q.argtypes = [vp, dp, i64]
        L.or_lsq.argtypes = [vp, i64, dp, i64, dp, i64, dp]
        L.or_lsq.restype = i64
        L.or_lsq_refined.argtypes = [vp, dp, i64, dp, dp, ctypes.c_int]
        L.or_lsq_refined.restype = i64
        L.or_max_threads.restype = ctypes.c_int
        L.or_tslu.argtypes = [i64, i64, dp, i64, i64, ip, ip, i64, i64, i64, ip, ip, ctypes.c_int,
                              ip, dp, i64, dp, i64]
        L.or_tslu.restype = i64
        L.or_cond1.argtypes = [i64, dp, i64]
        L.or_cond1.restype = ctypes.c_double
        L.or_cond1_est.argtypes = [i64, dp, i64]
        L.or_cond1_est.restype = ctypes.c_double
        L.or_cholesky.argtypes = [i64, dp, i64, dp, i64, ctypes.c_int]
        L.or_cholesky.restype = i64
        L.or_calu.argtypes = [i64, i64, dp, i64, i64, ctypes.c_int, ctypes.c_int, ip]
        L.or_calu.restype = i64
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _fortran(a) -> np.ndarray:
    return np.asfortranarray(np.array(a, dtype=np.float64, copy=True))


def max_threads() -> int:
    return int(lib().or_max_threads())


# --- single building blocks (Sec. 2.2 reflector / compact WY, Sec. 2.3 combine)

def larfg(alpha: float, x):
    """Householder reflector H = I - tau v v^T with H [alpha; x] = beta e_1
    (Sec. 2.2).  Returns (beta, v_tail, tau), v = [1; v_tail]."""
    x = np.array(x, dtype=np.float64, copy=True)
    a = ctypes.c_double(alpha)
    t = ctypes.c_double(0.0)
    lib().or_larfg(x.size, ctypes.byref(a), _dp(x), 1, ctypes.byref(t))
    return a.value, x, t.value


def geqrt(A):
    """Householder QR of one domain with its compact-WY T (Sec. 2.2).
    Returns (W, tau, T): R on/above the diagonal of W, reflectors below."""
    W = _fortran(A)
    r, n = W.shape
    tau = np.zeros(n)
    T = np.zeros((n, n), order="F")
    lib().or_geqrt(r, n, _dp(W), r, _dp(tau), _dp(T), n)
    return W, tau, T


def tpqrt(R1, R2):
    """Tree combine: QR of the stacked triangles [R1; R2] (Sec. 2.3).
    Returns (R, U, tau, T): U holds the reflector tails in its upper triangle."""
    A = _fortran(np.triu(R1))
    B = _fortran(np.triu(R2))
    n = A.shape[0]
    tau = np.zeros(n)
    T = np.zeros((n, n), order="F")
    lib().or_tpqrt(n, _dp(A), n, _dp(B), n, _dp(tau), _dp(T), n)
    return A, B, tau, T


def partition(m: int, n: int, mb: int):
    """Domain partition (Sec. 2.3): list of (row0, nrows)."""
    P = int(lib().or_partition(m, n, mb, None, None))
    if P < 1:
        raise ValueError("invalid partition arguments")
    r0 = np.zeros(P, dtype=np.int64)
    nr = np.zeros(P, dtype=np.int64)
    lib().or_partition(m, n, mb, _ip(r0), _ip(nr))
    return list(zip(r0.tolist(), nr.tolist()))


def partition_weighted(m: int, n: int, P: int, granule: int, weights=None):
    """Load-balanced partition (Sec. 3: rows per domain follow the
    processing power given to it): list of (row0, nrows) for P domains of
    integer powers `weights` (None = equal), in whole granules of `granule`
    rows, apportioned by largest remainders (ties to the lower index)."""
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.int64)
    if w is not None and w.shape != (P,):
        raise ValueError("one weight per domain")
    r0 = np.zeros(P, dtype=np.int64)
    nr = np.zeros(P, dtype=np.int64)
    got = int(lib().or_partition_weighted(m, n, P, granule, None if w is None else _ip(w), _ip(r0), _ip(nr)))
    if got < 1:
        raise ValueError("no such partition (a domain gets no granule or fewer than n rows)")
    return list(zip(r0.tolist(), nr.tolist()))


def tslu(A, parts, first: int, stage: int, tree: int = TREE_BINARY, sched=None, nthreads: int = 0):
    """LU with tournament pivoting (TSQR's tree applied to LU, the paper's
    conclusion): each domain (row0, nrows) of `parts` selects b pivot rows by
    partial-pivoting elimination over stages (its first `first` rows, then
    its selection stacked on the next `stage` rows), the domains' selections
    are combined along the tree, and A = L U with U the LU of A[ipiv] and
    l_i = a_i U^{-1}.  Returns (ipiv, L, U, info)."""
    A = _fortran(A)
    m, b = A.shape
    P = len(parts)
    if sched is None:
        sched = schedule(P, tree)
    r0 = np.array([p[0] for p in parts], dtype=np.int64)
    nr = np.array([p[1] for p in parts], dtype=np.int64)
    sl = np.array([s[0] for s in sched] or [0], dtype=np.int64)
    sr = np.array([s[1] for s in sched] or [0], dtype=np.int64)
    ipiv = np.zeros(b, dtype=np.int64)
    L = np.zeros((m, b), order="F")
    U = np.zeros((b, b), order="F")
    nt = nthreads if nthreads > 0 else max_threads()
    info = int(lib().or_tslu(m, b, _dp(A), m, P, _ip(r0), _ip(nr), first, stage, len(sched), _ip(sl),
                             _ip(sr), nt, _ip(ipiv), _dp(L), m, _dp(U), b))
    if info < 0:
        raise ValueError("oracle TSLU rejected its arguments")
    return ipiv, L, U, info


def cond1(R) -> float:
    """kappa_1(R) = ||R||_1 ||R^{-1}||_1 of an upper-triangular R, exactly
    (R^{-1} by back substitution); +inf for a zero diagonal."""
    R = _fortran(R)
    return float(lib().or_cond1(R.shape[0], _dp(R), R.shape[0]))


def cond1_est(R) -> float:
    """The cheap lower-bound estimate of kappa_1(R) (Hager 1984, Higham 1988)."""
    R = _fortran(R)
    return float(lib().or_cond1_est(R.shape[0], _dp(R), R.shape[0]))


def cholesky(A, nthreads: int = 0):
    """Cholesky factor of a symmetric positive definite A (the one-sided
    factorization the paper names beside QR and LU), from the definition
    column by column; only the lower triangle of A is read.  Returns (L,
    info): L lower triangular with zeros above, info = 0 or j + 1 for the
    first leading minor of order j + 1 that is not positive definite
    (columns 0..j-1 of L final, the rest zero)."""
    A = _fortran(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    L = np.zeros((n, n), order="F")
    nt = nthreads if nthreads > 0 else max_threads()
    info = int(lib().or_cholesky(n, _dp(A), max(n, 1), _dp(L), max(n, 1), nt))
    if info < 0:
        raise ValueError("oracle Cholesky rejected its arguments")
    return L, info


def calu(A, mb: int, tree: int = TREE_BINARY, nthreads: int = 0):
    """LU with tournament pivoting of an m x n matrix (m >= n; CALU, the LU
    counterpart of CAQR named in the conclusion): 64-column panels, each
    pivoted by TSLU over or_partition(m - k, b, mb) and the tree, the pivots
    applied as LAPACK-style row interchanges.  Returns (LU, ipiv, info) in
    dgetrf's layout: P A = L U with L unit lower (strictly below the
    diagonal of LU) and U upper, ipiv[i] = the row swapped with row i
    (0-based), info = 0 or the first j + 1 with U_jj == 0."""
    LU = _fortran(A)
    m, n = LU.shape
    ipiv = np.zeros(n, dtype=np.int64)
    nt = nthreads if nthreads > 0 else max_threads()
    info = int(lib().or_calu(m, n, _dp(LU), m, mb, tree, nt, _ip(ipiv)))
    if info < 0:
        raise ValueError("oracle CALU rejected its arguments")
    return LU, ipiv, info


def schedule(P: int, tree: int):
    """Reduction-tree schedule (Sec. 2.3): list of (left, right) combines."""
    sl = np.zeros(max(P - 1, 1), dtype=np.int64)
    sr = np.zeros(max(P - 1, 1), dtype=np.int64)
    cnt = int(lib().or_schedule(P, tree, _ip(sl), _ip(sr)))
    return list(zip(sl[:cnt].tolist(), sr[:cnt].tolist()))


def hierarchical_schedule(group):
    """Grid-tuned reduction tree (Sec. 2.3, Fig. 2; Sec. 3): domain d
    belongs to cluster group[d]; the domains of each cluster are reduced by a
    binary tree over its members in increasing order (the result in the
    smallest), then the cluster roots by a binary tree in increasing order
    of their indices.  Returns the (left, right) combines, cluster by
    cluster, then across clusters; only one combine per cluster boundary
    of that last tree, G - 1 in all, joins two clusters."""
    members = {}
    for d, g in enumerate(group):
        members.setdefault(g, []).append(d)
    sched = []
    roots = []
    for g in sorted(members, key=lambda g: members[g][0]):
        mem = members[g]
        sched += [(mem[l], mem[r]) for l, r in schedule(len(mem), TREE_BINARY)]
        roots.append(mem[0])
    sched += [(roots[l], roots[r]) for l, r in schedule(len(roots), TREE_BINARY)]
    return sched


class TSQR:
    """TSQR factorization of an m x n matrix (Sec. 2.3) held by the oracle."""

    def __init__(self, A, mb: int = 0, tree: int = TREE_BINARY, nthreads: int = 0,
                 sched=None, parts=None):
        """mb: rows per domain; parts: an explicit partition, a list of
        (row0, nrows) (e.g. from partition_weighted), in place of mb."""
        A = _fortran(A)
        self.m, self.n = A.shape
        self.mb = mb
        nt = nthreads if nthreads > 0 else max_threads()
        if parts is not None:
            P = len(parts)
            if sched is None:
                sched = schedule(P, tree)
            r0 = np.array([p[0] for p in parts], dtype=np.int64)
            nr = np.array([p[1] for p in parts], dtype=np.int64)
            sl = np.array([s[0] for s in sched] or [0], dtype=np.int64)
            sr = np.array([s[1] for s in sched] or [0], dtype=np.int64)
            h = lib().or_factor_parts(self.m, self.n, _dp(A), self.m, P, _ip(r0), _ip(nr),
                                      len(sched), _ip(sl), _ip(sr), nt)
        elif sched is None:
            h = lib().or_factor(self.m, self.n, _dp(A), self.m, mb, tree, nt)
        else:
            sl = np.array([s[0] for s in sched], dtype=np.int64)
            sr = np.array([s[1] for s in sched], dtype=np.int64)
            if len(sched) == 0:
                sl = np.zeros(1, dtype=np.int64)
                sr = np.zeros(1, dtype=np.int64)
            h = lib().or_factor_sched(self.m, self.n, _dp(A), self.m, mb, len(sched),
                                      _ip(sl), _ip(sr), nt)
        if not h:
            raise ValueError("oracle factor rejected its arguments")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_free(h)
            self._h = None

    @property
    def P(self) -> int:
        return int(lib().or_num_domains(self._h))

    def R(self) -> np.ndarray:
        R = np.zeros((self.n, self.n), order="F")
        lib().or_get_r(self._h, _dp(R), self.n)
        return R

    def leaf(self):
        W = np.zeros((self.m, self.n), order="F")
        tau = np.zeros((self.P, self.n))
        T = np.zeros((self.P, self.n, self.n))
        lib().or_get_leaf(self._h, _dp(W), _dp(tau), _dp(T))
        return W, tau, T

    def apply_qt(self, B) -> np.ndarray:
        B = _fortran(B)
        if B.ndim == 1:
            B = B.reshape(-1, 1, order="F")
        lib().or_apply_qt(self._h, B.shape[1], _dp(B), self.m)
        return B

    def form_q(self) -> np.ndarray:
        Q = np.zeros((self.m, self.n), order="F")
        lib().or_form_q(self._h, _dp(Q), self.m)
        return Q

    def lsq(self, B):
        """Returns (X, resid, info); info = j+1 for the first zero R_jj."""
        B = _fortran(B)
        if B.ndim == 1:
            B = B.reshape(-1, 1, order="F")
        k = B.shape[1]
        X = np.zeros((self.n, k), order="F")
        res = np.zeros(k)
        info = int(lib().or_lsq(self._h, k, _dp(B), self.m, _dp(X), self.n, _dp(res)))
        return X, res, info

    def lsq_refined(self, A, b, maxit: int = 30):
        """Least-squares reference refined with binary128 residuals."""
        A = _fortran(A)
        b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).ravel())
        x = np.zeros(self.n)
        it = int(lib().or_lsq_refined(self._h, _dp(A), self.m, _dp(b), _dp(x), maxit))
        if it < 0:
            raise np.linalg.LinAlgError("singular R")
        return x, it


def block_orth(V, W, mb: int, tree: int = TREE_BINARY):
    """One step of block orthogonalisation as block-iterative methods use
    TSQR (Scope section and Sec. 6 of the paper: TSQR generates an
    orthogonal basis stably): two passes of block classical Gram-Schmidt
    against the orthonormal V (NumPy products in FP64), then TSQR of the
    projected block.  Returns (Q, H, R) with W = V H + Q R."""
    W = np.array(W, dtype=np.float64, copy=True)
    m, b = W.shape
    if V is None or V.shape[1] == 0:
        H = np.zeros((0, b))
    else:
        V = np.asarray(V, dtype=np.float64)
        H1 = V.T @ W
        W = W - V @ H1
        H2 = V.T @ W
        W = W - V @ H2
        H = H1 + H2
    f = TSQR(W, mb=mb, tree=tree)
    return f.form_q(), H, f.R()

