"""MI355X-native TSQR (Agullo et al., arXiv 0912.2572, Sec. 2.3).

Thin Python binding over the C ABI of ``libtsqr.so`` (see include/tsqr.h):
argument marshalling only.  Every step of the factorization, the Q^T / Q
applications, the thin Q and least squares runs in the library's HIP kernels
for gfx950; PyTorch provides device memory and the stream.  There is no CPU
fallback: if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtsqr.so")

TREE_FLAT = 0
TREE_BINARY = 2
TREE_QUAD = 4
TREE_XCD = 8
F64 = 0
MIXED = 1

ERR_WORKSPACE = -900
ERR_STATE = -901
ERR_UNSUPPORTED = -902


class Opts(ctypes.Structure):
    _fields_ = [
        ("row_block", ctypes.c_int64),
        ("tree", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("keep_q", ctypes.c_int32),
        ("lsq_max_rhs", ctypes.c_int32),
        ("refine_max_iter", ctypes.c_int32),
        ("domains", ctypes.c_int32),
        ("refine_tol", ctypes.c_double),
        ("route_kappa", ctypes.c_double),
        ("domain_weights", ctypes.POINTER(ctypes.c_int64)),
        ("num_weights", ctypes.c_int64),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("n_max", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("row_block", ctypes.c_int64),
        ("tree", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("prec", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("A", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("b", ctypes.c_void_p),
        ("R", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("resid", ctypes.c_void_p),
        ("info", ctypes.c_void_p),
    ]


BATCH_DEFAULT_ROW_BLOCK = 4096


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("streams", ctypes.c_int32),
        ("max_inflight", ctypes.c_int32),
        ("cache", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("tree", ctypes.c_int32),
        ("bypass_ms", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("route_kappa", ctypes.c_double),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("matrix_id", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("X", ctypes.c_void_p),
        ("resid", ctypes.c_void_p),
        ("info", ctypes.c_void_p),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("cache_hits", ctypes.c_int64),
        ("evictions", ctypes.c_int64),
        ("bytes_in_use", ctypes.c_size_t),
        ("bytes_peak", ctypes.c_size_t),
        ("busy_seconds", ctypes.c_double),
        ("byte_seconds", ctypes.c_double),
    ]

_lib = None


def lib():
    """The loaded libtsqr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with `python -m paper_0912_2572_amd.build`"
            )
        L = ctypes.CDLL(_LIB_PATH)
        i64, i32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
        op = ctypes.POINTER(Opts)
        L.tsqr_default_opts.argtypes = [op]
        L.tsqr_default_opts.restype = None
        L.tsqr_workspace_bytes.argtypes = [i64, i64, op]
        L.tsqr_workspace_bytes.restype = sz
        L.tsqr_factor.argtypes = [i64, i64, vp, i64, op, vp, sz, vp, ctypes.POINTER(vp)]
        L.tsqr_get_r.argtypes = [vp, vp, i64, vp]
        L.tsqr_apply_qt.argtypes = [vp, i64, vp, i64, vp]
        L.tsqr_apply_q.argtypes = [vp, i64, vp, i64, vp]
        L.tsqr_form_q.argtypes = [vp, vp, i64, vp]
        L.tsqr_lsq_solve.argtypes = [vp, vp, i64, i64, vp, i64, vp, i64, vp, vp, vp]
        L.tsqr_factor_solve.argtypes = [i64, i64, vp, i64, op, vp, sz, i64, vp, i64, vp, i64, vp, vp, vp,
                                        i64, vp, ctypes.POINTER(vp)]
        L.tsqr_last_refine_iters.argtypes = [vp, vp]
        L.tsqr_lsq_backward_error.argtypes = [vp, i64, vp, vp]
        L.tsqr_block_orth_workspace_bytes.argtypes = [i64, i64, i64, op]
        L.tsqr_block_orth_workspace_bytes.restype = sz
        L.tsqr_block_orth.argtypes = [i64, i64, vp, i64, i64, vp, i64, vp, i64, vp, i64, op, vp, sz, vp]
        L.tsqr_block_orth.restype = ctypes.c_int
        L.tsqr_factor_solve_noalloc.argtypes = [i64, i64, vp, i64, op, i64, vp, i64, vp, i64, vp, vp, vp, i64,
                                                vp, i64, vp]
        L.tsqr_factor_solve_noalloc.restype = ctypes.c_int
        L.tsqr_plan_info.argtypes = [i64, i64, op, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     ctypes.POINTER(i64)]
        L.tsqr_tslu_workspace_bytes.argtypes = [i64, i64, op]
        L.tsqr_tslu_workspace_bytes.restype = sz
        L.tsqr_tslu.argtypes = [i64, i64, vp, i64, op, vp, sz, vp, i64, vp, i64, vp, vp, vp]
        L.tsqr_tslu.restype = ctypes.c_int
        L.tsqr_cond_estimate.argtypes = [vp, vp, vp]
        L.tsqr_cholesky.argtypes = [i64, vp, i64, vp, vp]
        L.tsqr_calu_workspace_bytes.argtypes = [i64, i64, op]
        L.tsqr_calu_workspace_bytes.restype = sz
        L.tsqr_calu.argtypes = [i64, i64, vp, i64, op, vp, sz, vp, vp, vp]
        L.tsqr_calu.restype = ctypes.c_int
        L.tsqr_cholesky.restype = ctypes.c_int
        L.tsqr_cond_estimate.restype = ctypes.c_int
        L.tsqr_route_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        L.tsqr_route_info.restype = ctypes.c_int
        L.tsqr_partition.argtypes = [i64, i64, op, ctypes.POINTER(i64), ctypes.POINTER(i64), i64]
        L.tsqr_partition.restype = i64
        L.tsqr_tree_schedule.argtypes = [i64, ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(i64), i64]
        L.tsqr_tree_schedule.restype = i64
        L.tsqr_prof_enable.argtypes = [ctypes.c_int]
        L.tsqr_prof_enable.restype = ctypes.c_int
        L.tsqr_prof_only.argtypes = [ctypes.c_char_p]
        L.tsqr_prof_only.restype = ctypes.c_int
        L.tsqr_prof_query.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
        L.tsqr_prof_query.restype = ctypes.c_int
        L.tsqr_free.argtypes = [vp]
        L.tsqr_strerror.argtypes = [ctypes.c_int]
        L.tsqr_strerror.restype = ctypes.c_char_p
        bip, tep = ctypes.POINTER(BatchItem), ctypes.POINTER(TuneEntry)
        L.tsqr_batch_workspace_bytes.argtypes = [ctypes.c_int, bip, tep, ctypes.c_int]
        L.tsqr_batch_workspace_bytes.restype = sz
        L.tsqr_batch_create.argtypes = [ctypes.c_int, bip, tep, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        vp, sz, vp, ctypes.POINTER(vp)]
        L.tsqr_batch_bad_item.argtypes = []
        L.tsqr_batch_run.argtypes = [vp, ctypes.c_int, vp]
        L.tsqr_batch_plan.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                      ctypes.POINTER(i64)]
        L.tsqr_batch_launches.argtypes = [vp]
        L.tsqr_batch_free.argtypes = [vp]
        L.tsqr_autotune.argtypes = [ctypes.c_int, bip, ctypes.c_int, vp, sz, vp, tep, ctypes.c_int]
        sop = ctypes.POINTER(ServerOpts)
        L.tsqr_server_default_opts.argtypes = [sop]
        L.tsqr_server_default_opts.restype = None
        L.tsqr_server_create.argtypes = [sop, ctypes.POINTER(vp)]
        L.tsqr_server_submit.argtypes = [vp, ctypes.POINTER(Request)]
        L.tsqr_server_submit.restype = i64
        L.tsqr_server_progress.argtypes = [vp, ctypes.c_int]
        L.tsqr_server_status.argtypes = [vp, i64]
        L.tsqr_server_times.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.tsqr_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.tsqr_server_free.argtypes = [vp]
        L.tsqr_server_now.argtypes = []
        L.tsqr_server_now.restype = ctypes.c_double
        for name in ("tsqr_server_create", "tsqr_server_progress", "tsqr_server_status",
                     "tsqr_server_times", "tsqr_server_get_stats", "tsqr_server_free"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("tsqr_factor", "tsqr_get_r", "tsqr_apply_qt", "tsqr_apply_q", "tsqr_form_q",
                     "tsqr_lsq_solve", "tsqr_last_refine_iters", "tsqr_lsq_backward_error", "tsqr_plan_info", "tsqr_free",
                     "tsqr_batch_create", "tsqr_batch_bad_item", "tsqr_batch_run", "tsqr_batch_plan",
                     "tsqr_batch_launches", "tsqr_batch_free", "tsqr_autotune"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class TSQRError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what} failed: {code} ({lib().tsqr_strerror(code).decode()})")


def _check(code: int, what: str):
    if code != 0:
        raise TSQRError(code, what)


def opts(row_block: int = 0, tree: int = TREE_BINARY, prec: int = F64, keep_q: bool = True,
         lsq_max_rhs: int = 8, refine_max_iter: int = 30, refine_tol: float = 1e-14,
         domains: int = 0, route_kappa: float = 0.0, weights=None) -> Opts:
    """domains > 0 (or -1: one per resident leaf workgroup) selects the
    load-balanced partition in place of row_block; weights (one integer
    power >= 1 per domain) the weighted one; route_kappa > 0 sends a
    mixed-precision solve whose R is estimated worse conditioned to FP64
    (see tsqr.h)."""
    o = Opts()
    lib().tsqr_default_opts(ctypes.byref(o))
    o.row_block = row_block
    o.domains = domains
    o.route_kappa = route_kappa
    if weights is not None:
        w = (ctypes.c_int64 * len(weights))(*[int(x) for x in weights])
        o._weights = w          # keeps the array alive as long as the options
        o.domain_weights = ctypes.cast(w, ctypes.POINTER(ctypes.c_int64))
        o.num_weights = len(weights)
    o.tree = tree
    o.prec = prec
    o.keep_q = 1 if keep_q else 0
    o.lsq_max_rhs = lsq_max_rhs
    o.refine_max_iter = refine_max_iter
    o.refine_tol = refine_tol
    return o


def workspace_bytes(m: int, n: int, o: Opts | None = None) -> int:
    return int(lib().tsqr_workspace_bytes(m, n, ctypes.byref(o) if o is not None else None))


def plan_info(m: int, n: int, o: Opts | None = None):
    P, c, npan = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().tsqr_plan_info(m, n, ctypes.byref(o) if o is not None else None,
                                ctypes.byref(P), ctypes.byref(c), ctypes.byref(npan)), "tsqr_plan_info")
    return P.value, c.value, npan.value


def partition(m: int, n: int, o: Opts | None = None):
    """The library's domains of the first panel as (row0, nrows) pairs."""
    op = ctypes.byref(o) if o is not None else None
    P = int(lib().tsqr_partition(m, n, op, None, None, 0))
    if P < 0:
        raise TSQRError(P, "tsqr_partition")
    r0 = (ctypes.c_int64 * P)()
    nr = (ctypes.c_int64 * P)()
    lib().tsqr_partition(m, n, op, r0, nr, P)
    return [(r0[i], nr[i]) for i in range(P)]


def tree_schedule(P: int, tree: int):
    """The library's reduction tree as (left, right) combines in order."""
    cap = max(P - 1, 1)
    left = (ctypes.c_int64 * cap)()
    right = (ctypes.c_int64 * cap)()
    cnt = int(lib().tsqr_tree_schedule(P, tree, left, right, cap))
    if cnt < 0:
        raise ValueError("invalid tree arguments")
    return [(left[i], right[i]) for i in range(cnt)]


def prof_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events (see tsqr.h)."""
    lib().tsqr_prof_enable(1 if on else 0)


def prof_only(tag: str | None) -> None:
    """Time only the kernels tagged `tag` (None: all), see tsqr.h."""
    lib().tsqr_prof_only(tag.encode() if tag else None)


def prof_query() -> dict:
    """{kernel name: (launches, total ms)} of the launches timed so far."""
    out = {}
    i = 0
    while True:
        name = ctypes.c_char_p()
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        if lib().tsqr_prof_query(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)) != 0:
            break
        out[name.value.decode()] = (cnt.value, ms.value)
        i += 1
    return out


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _col_major(t: torch.Tensor, rows: int, name: str):
    """(pointer, leading dimension) of a column-major float64 device matrix."""
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr(), max(rows, t.shape[0])
    if t.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (use .t().contiguous().t() or "
                         "torch.empty((n, m)).t())")
    return t.data_ptr(), t.stride(1) if t.shape[1] > 1 else max(t.stride(1), t.shape[0])


def empty_colmajor(m: int, n: int, device="cuda", dtype=torch.float64) -> torch.Tensor:
    return torch.empty((n, m), device=device, dtype=dtype).t()


def to_colmajor(x, device="cuda") -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.dim() == 1:
        return t.to(device).contiguous()
    return t.t().contiguous().t().to(device) if t.device.type == "cpu" else t.t().contiguous().t()


class Factors:
    """One TSQR factorization living in a caller-owned device workspace."""

    def __init__(self, A: torch.Tensor, o: Opts | None = None, work: torch.Tensor | None = None,
                 stream=None):
        m, n = A.shape
        self.m, self.n = m, n
        self.opts = o if o is not None else opts()
        need = workspace_bytes(m, n, self.opts)
        if need == 0:
            raise ValueError(f"invalid problem {m} x {n} for the given options")
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=A.device)
        self.work = work
        pa, lda = _col_major(A, m, "A")
        h = ctypes.c_void_p()
        _check(lib().tsqr_factor(m, n, ctypes.c_void_p(pa), lda, ctypes.byref(self.opts),
                                 ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(stream),
                                 ctypes.byref(h)), "tsqr_factor")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tsqr_free(h)
            self._h = None

    def R(self, stream=None) -> torch.Tensor:
        R = empty_colmajor(self.n, self.n, device=self.work.device)
        _check(lib().tsqr_get_r(self._h, ctypes.c_void_p(R.data_ptr()), self.n, _stream(stream)),
               "tsqr_get_r")
        return R

    def apply_qt_(self, B: torch.Tensor, stream=None) -> torch.Tensor:
        k = 1 if B.dim() == 1 else B.shape[1]
        pb, ldb = _col_major(B, self.m, "B")
        _check(lib().tsqr_apply_qt(self._h, k, ctypes.c_void_p(pb), ldb, _stream(stream)),
               "tsqr_apply_qt")
        return B

    def apply_q_(self, B: torch.Tensor, stream=None) -> torch.Tensor:
        k = 1 if B.dim() == 1 else B.shape[1]
        pb, ldb = _col_major(B, self.m, "B")
        _check(lib().tsqr_apply_q(self._h, k, ctypes.c_void_p(pb), ldb, _stream(stream)),
               "tsqr_apply_q")
        return B

    def form_q(self, Q: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if Q is None:
            Q = empty_colmajor(self.m, self.n, device=self.work.device)
        pq, ldq = _col_major(Q, self.m, "Q")
        _check(lib().tsqr_form_q(self._h, ctypes.c_void_p(pq), ldq, _stream(stream)), "tsqr_form_q")
        return Q

    def lsq(self, B: torch.Tensor, A: torch.Tensor | None = None, X: torch.Tensor | None = None,
            resid: torch.Tensor | None = None, info: torch.Tensor | None = None, stream=None):
        """Least squares through the factors.  Returns device tensors
        (X, resid, info); info is an int32 scalar tensor."""
        k = 1 if B.dim() == 1 else B.shape[1]
        dev = self.work.device
        if X is None:
            X = empty_colmajor(self.n, k, device=dev)
        if resid is None:
            resid = torch.empty(k, dtype=torch.float64, device=dev)
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        pb, ldb = _col_major(B, self.m, "B")
        px, ldx = _col_major(X, self.n, "X")
        pa, lda = (0, self.m) if A is None else _col_major(A, self.m, "A")
        _check(lib().tsqr_lsq_solve(self._h, ctypes.c_void_p(pa), lda, k, ctypes.c_void_p(pb), ldb,
                                    ctypes.c_void_p(px), ldx, ctypes.c_void_p(resid.data_ptr()),
                                    ctypes.c_void_p(info.data_ptr()), _stream(stream)),
               "tsqr_lsq_solve")
        return X, resid, info

    def backward_error(self, k: int, stream=None) -> torch.Tensor:
        """Backward-error bounds (device, k doubles) of the last mixed-precision
        least-squares solve on this factor."""
        eta = torch.empty(k, dtype=torch.float64, device=self.work.device)
        _check(lib().tsqr_lsq_backward_error(self._h, k, ctypes.c_void_p(eta.data_ptr()), _stream(stream)),
               "tsqr_lsq_backward_error")
        return eta

    def last_refine_iters(self, stream=None) -> int:
        return int(lib().tsqr_last_refine_iters(self._h, _stream(stream)))

    def cond_estimate(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """kappa_1(R) estimate (tsqr_cond_estimate) as a one-element device tensor."""
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.work.device)
        _check(lib().tsqr_cond_estimate(self._h, ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "tsqr_cond_estimate")
        return out

    def route_info(self):
        """(precision of the reflectors now, condition estimate that routed it or 0)."""
        prec, kap = ctypes.c_int32(), ctypes.c_double()
        _check(lib().tsqr_route_info(self._h, ctypes.byref(prec), ctypes.byref(kap)), "tsqr_route_info")
        return prec.value, kap.value


def factor_solve(A: torch.Tensor, B: torch.Tensor, o: Opts | None = None, work: torch.Tensor | None = None,
                 X: torch.Tensor | None = None, resid: torch.Tensor | None = None,
                 info: torch.Tensor | None = None, Q: torch.Tensor | None = None, stream=None):
    """Factor A, solve min ||A x - b|| for the columns of B and, if Q is
    given, write the thin Q, in one call (tsqr_factor_solve).  Returns
    (Factors, X, resid, info)."""
    m, n = A.shape
    k = 1 if B.dim() == 1 else B.shape[1]
    o = o if o is not None else opts()
    dev = A.device
    need = workspace_bytes(m, n, o)
    if need == 0:
        raise ValueError(f"invalid problem {m} x {n} for the given options")
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    if X is None:
        X = empty_colmajor(n, k, device=dev)
    if resid is None:
        resid = torch.empty(k, dtype=torch.float64, device=dev)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=dev)
    pa, lda = _col_major(A, m, "A")
    pb, ldb = _col_major(B, m, "B")
    px, ldx = _col_major(X, n, "X")
    pq, ldq = (0, m) if Q is None else _col_major(Q, m, "Q")
    h = ctypes.c_void_p()
    _check(lib().tsqr_factor_solve(m, n, ctypes.c_void_p(pa), lda, ctypes.byref(o),
                                   ctypes.c_void_p(work.data_ptr()), work.numel(), k, ctypes.c_void_p(pb), ldb,
                                   ctypes.c_void_p(px), ldx, ctypes.c_void_p(resid.data_ptr()),
                                   ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(pq), ldq, _stream(stream),
                                   ctypes.byref(h)), "tsqr_factor_solve")
    F = Factors.__new__(Factors)
    F.m, F.n, F.opts, F.work, F._h = m, n, o, work, h
    return F, X, resid, info


def tslu(A: torch.Tensor, o: Opts | None = None, work: torch.Tensor | None = None, L: torch.Tensor | None = None,
         U: torch.Tensor | None = None, stream=None):
    """LU with tournament pivoting over the TSQR partition and tree
    (tsqr_tslu): returns (ipiv, L, U, info) with A = L U, ipiv the pivot rows
    of A in order and L a row permutation of a unit lower trapezoidal matrix."""
    m, b = A.shape
    o = o if o is not None else opts()
    dev = A.device
    need = int(lib().tsqr_tslu_workspace_bytes(m, b, ctypes.byref(o)))
    if need == 0:
        raise ValueError(f"invalid TSLU problem {m} x {b} for the given options")
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    if L is None:
        L = empty_colmajor(m, b, device=dev)
    if U is None:
        U = empty_colmajor(b, b, device=dev)
    ipiv = torch.empty(b, dtype=torch.int64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    pa, lda = _col_major(A, m, "A")
    pl, ldl = _col_major(L, m, "L")
    pu, ldu = _col_major(U, b, "U")
    _check(lib().tsqr_tslu(m, b, ctypes.c_void_p(pa), lda, ctypes.byref(o), ctypes.c_void_p(work.data_ptr()),
                           work.numel(), ctypes.c_void_p(pl), ldl, ctypes.c_void_p(pu), ldu,
                           ctypes.c_void_p(ipiv.data_ptr()), ctypes.c_void_p(info.data_ptr()), _stream(stream)),
           "tsqr_tslu")
    return ipiv, L, U, info


def calu(A: torch.Tensor, o: Opts | None = None, work: torch.Tensor | None = None,
         ipiv: torch.Tensor | None = None, info: torch.Tensor | None = None, stream=None):
    """In-place LU with tournament pivoting (tsqr_calu) of a column-major
    m x n A (m >= n): A becomes dgetrf's packed L\\U with P A = L U.
    Returns (ipiv, info): ipiv[i] the row interchanged with row i (0-based)."""
    m, n = A.shape
    o = o if o is not None else opts()
    dev = A.device
    need = int(lib().tsqr_calu_workspace_bytes(m, n, ctypes.byref(o)))
    if need == 0:
        raise ValueError(f"invalid CALU problem {m} x {n} for the given options")
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    if ipiv is None:
        ipiv = torch.empty(n, dtype=torch.int64, device=dev)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=dev)
    pa, lda = _col_major(A, m, "A")
    _check(lib().tsqr_calu(m, n, ctypes.c_void_p(pa), lda, ctypes.byref(o), ctypes.c_void_p(work.data_ptr()),
                           work.numel(), ctypes.c_void_p(ipiv.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                           _stream(stream)), "tsqr_calu")
    return ipiv, info


def cholesky(A: torch.Tensor, info: torch.Tensor | None = None, stream=None):
    """In-place Cholesky factorization A = L L^T of a symmetric positive
    definite matrix (tsqr_cholesky): reads the lower triangle of the
    column-major A, overwrites it with L and leaves the strict upper
    triangle alone.  Returns the device info word (0, or the order of the
    first leading minor that is not positive definite)."""
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n:
        raise ValueError("A must be square")
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    pa, lda = _col_major(A, n, "A") if n > 0 else (0, 1)
    _check(lib().tsqr_cholesky(n, ctypes.c_void_p(pa), lda, ctypes.c_void_p(info.data_ptr()), _stream(stream)),
           "tsqr_cholesky")
    return info


NOALLOC_SCRATCH_BYTES = 64 << 20


def factor_solve_noalloc(A: torch.Tensor, B: torch.Tensor, o: Opts | None = None, X: torch.Tensor | None = None,
                         resid: torch.Tensor | None = None, info: torch.Tensor | None = None,
                         Q: torch.Tensor | None = None, R: torch.Tensor | None = None, stream=None):
    """tsqr_factor_solve_noalloc: factor, least squares and (if given) the
    thin Q and R with the library's static device scratch as the workspace
    (no device allocation inside the call; the outputs are the caller's).
    Returns (X, resid, info)."""
    m, n = A.shape
    k = 1 if B.dim() == 1 else B.shape[1]
    o = o if o is not None else opts()
    dev = A.device
    if X is None:
        X = empty_colmajor(n, k, device=dev)
    if resid is None:
        resid = torch.empty(k, dtype=torch.float64, device=dev)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=dev)
    pa, lda = _col_major(A, m, "A")
    pb, ldb = _col_major(B, m, "B")
    px, ldx = _col_major(X, n, "X")
    pq, ldq = (0, m) if Q is None else _col_major(Q, m, "Q")
    pr, ldr = (0, n) if R is None else _col_major(R, n, "R")
    _check(lib().tsqr_factor_solve_noalloc(m, n, ctypes.c_void_p(pa), lda, ctypes.byref(o), k, ctypes.c_void_p(pb),
                                           ldb, ctypes.c_void_p(px), ldx, ctypes.c_void_p(resid.data_ptr()),
                                           ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(pq), ldq,
                                           ctypes.c_void_p(pr), ldr, _stream(stream)),
           "tsqr_factor_solve_noalloc")
    return X, resid, info


def block_orth(V: torch.Tensor | None, W: torch.Tensor, o: Opts | None = None, H: torch.Tensor | None = None,
               R: torch.Tensor | None = None, work: torch.Tensor | None = None, stream=None):
    """tsqr_block_orth: W <- Q with W_in = V H + Q R, [V Q] orthonormal (V may
    be None for the first block).  W is overwritten; returns (W, H, R)."""
    m, b = W.shape
    nv = 0 if V is None else V.shape[1]
    o = o if o is not None else opts()
    dev = W.device
    need = int(lib().tsqr_block_orth_workspace_bytes(m, nv, b, ctypes.byref(o)))
    if need == 0:
        raise ValueError(f"block_orth out of scope: m={m} nv={nv} b={b}")
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    if H is None and nv > 0:
        H = empty_colmajor(nv, b, device=dev)
    if R is None:
        R = empty_colmajor(b, b, device=dev)
    pv, ldv = (0, m) if V is None else _col_major(V, m, "V")
    pw, ldw = _col_major(W, m, "W")
    ph, ldh = (0, max(nv, 1)) if H is None else _col_major(H, nv, "H")
    pr, ldr = _col_major(R, b, "R")
    _check(lib().tsqr_block_orth(m, nv, ctypes.c_void_p(pv), ldv, b, ctypes.c_void_p(pw), ldw, ctypes.c_void_p(ph),
                                 ldh, ctypes.c_void_p(pr), ldr, ctypes.byref(o), ctypes.c_void_p(work.data_ptr()),
                                 work.numel(), _stream(stream)), "tsqr_block_orth")
    return W, H, R


def factor(A: torch.Tensor, **kw) -> Factors:
    work = kw.pop("work", None)
    stream = kw.pop("stream", None)
    return Factors(A, opts(**kw), work=work, stream=stream)


# ---------------------------------------------------------------------------
# Batched path


def tune_table(entries) -> tuple:
    """(ctypes array, count) from a list of dicts {n_max, prec, row_block, tree}."""
    if not entries:
        return None, 0
    arr = (TuneEntry * len(entries))()
    for i, e in enumerate(entries):
        arr[i].n_max, arr[i].prec = int(e["n_max"]), int(e["prec"])
        arr[i].row_block, arr[i].tree = int(e["row_block"]), int(e["tree"])
    return arr, len(entries)


def _items(As, bs, precs, outs):
    cnt = len(As)
    arr = (BatchItem * cnt)()
    for i in range(cnt):
        A = As[i]
        m, n = A.shape
        pa, lda = _col_major(A, m, "A")
        arr[i].m, arr[i].n, arr[i].prec = m, n, int(precs[i])
        arr[i].A, arr[i].lda = pa, lda
        if outs is not None:
            R, x, res, info = outs[i]
            arr[i].b = bs[i].data_ptr()
            arr[i].R, arr[i].x = R.data_ptr(), x.data_ptr()
            arr[i].resid, arr[i].info = res.data_ptr(), info.data_ptr()
    return arr


class Batch:
    """Many independent least-squares problems (n <= 64, one right-hand side
    each), factored and solved together by tsqr_batch_run.  Outputs per
    matrix: R (n x n), x (n), resid (1), info (1), all device tensors."""

    def __init__(self, As, bs, precs, tune=None, refine_sweeps: int = 4, refine_tol: float = 1e-14,
                 work: torch.Tensor | None = None, stream=None):
        dev = As[0].device
        self.count = len(As)
        self.As, self.bs = As, [b.reshape(-1).contiguous() for b in bs]
        self.outs = []
        for A in As:
            n = A.shape[1]
            self.outs.append((torch.empty((n, n), dtype=torch.float64, device=dev),
                              torch.empty(n, dtype=torch.float64, device=dev),
                              torch.empty(1, dtype=torch.float64, device=dev),
                              torch.empty(1, dtype=torch.int32, device=dev)))
        self._items = _items(As, self.bs, precs, self.outs)
        self._tune, ntune = tune_table(tune)
        need = lib().tsqr_batch_workspace_bytes(self.count, self._items, self._tune, ntune)
        if need == 0:
            raise ValueError(f"invalid batch item {lib().tsqr_batch_bad_item()}")
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=dev)
        self.work = work
        h = ctypes.c_void_p()
        _check(lib().tsqr_batch_create(self.count, self._items, self._tune, ntune, refine_sweeps,
                                       refine_tol, ctypes.c_void_p(work.data_ptr()), work.numel(),
                                       _stream(stream), ctypes.byref(h)), "tsqr_batch_create")
        self._h = h

    def run(self, use_graph: bool = True, stream=None):
        _check(lib().tsqr_batch_run(self._h, 1 if use_graph else 0, _stream(stream)), "tsqr_batch_run")

    def plan(self, i: int):
        mb, tr, P = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().tsqr_batch_plan(self._h, i, ctypes.byref(mb), ctypes.byref(tr), ctypes.byref(P)),
               "tsqr_batch_plan")
        return mb.value, tr.value, P.value

    def launches(self) -> int:
        return int(lib().tsqr_batch_launches(self._h))

    def R(self, i):
        # the library writes R column-major with leading dimension n
        return self.outs[i][0].t()

    def x(self, i):
        return self.outs[i][1]

    def resid(self, i):
        return self.outs[i][2]

    def info(self, i):
        return self.outs[i][3]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tsqr_batch_free(h)
            self._h = None


def batch_workspace_bytes(shapes, precs, tune=None) -> int:
    """Workspace for a batch of (m, n) shapes (tune None: the autotuning
    space's maximum)."""
    cnt = len(shapes)
    arr = (BatchItem * cnt)()
    for i, (m, n) in enumerate(shapes):
        arr[i].m, arr[i].n, arr[i].prec, arr[i].lda = m, n, int(precs[i]), m
    t, nt = tune_table(tune)
    return int(lib().tsqr_batch_workspace_bytes(cnt, arr, t, nt))


def autotune(As, bs, precs, reps: int = 2, stream=None):
    """Runs the C++ autotuner on this batch; returns the table as a list of
    dicts (save it as JSON to reuse it)."""
    dev = As[0].device
    outs = [(torch.empty((A.shape[1], A.shape[1]), dtype=torch.float64, device=dev),
             torch.empty(A.shape[1], dtype=torch.float64, device=dev),
             torch.empty(1, dtype=torch.float64, device=dev),
             torch.empty(1, dtype=torch.int32, device=dev)) for A in As]
    bs = [b.reshape(-1).contiguous() for b in bs]
    items = _items(As, bs, precs, outs)
    need = lib().tsqr_batch_workspace_bytes(len(As), items, None, 0)
    if need == 0:
        raise ValueError(f"invalid batch item {lib().tsqr_batch_bad_item()}")
    work = torch.empty(need, dtype=torch.uint8, device=dev)
    cap = 16
    out = (TuneEntry * cap)()
    rc = lib().tsqr_autotune(len(As), items, reps, ctypes.c_void_p(work.data_ptr()), work.numel(),
                             _stream(stream), out, cap)
    if rc < 0:
        raise TSQRError(rc, "tsqr_autotune")
    return [{"n_max": out[i].n_max, "prec": out[i].prec, "row_block": out[i].row_block,
             "tree": out[i].tree} for i in range(rc)]


# ---------------------------------------------------------------------------
# Serving


def _host_colmajor_ptr(t: torch.Tensor, name: str) -> int:
    if t.device.type != "cpu" or t.dtype not in (torch.float64, torch.int32):
        raise TypeError(f"{name} must be a host float64/int32 tensor")
    if t.dim() == 2 and not (t.stride(0) == 1 and (t.shape[1] == 1 or t.stride(1) == t.shape[0])):
        raise ValueError(f"{name} must be dense column-major")
    if t.dim() == 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


class Server:
    """Least-squares request server (tsqr_server_* in the C ABI).  Host
    tensors passed to submit() must stay alive until the request is done;
    the server keeps references to them."""

    def __init__(self, hbm_budget: int = 8 << 30, streams: int = 4, max_inflight: int = 16,
                 cache: bool = True, prec: int = F64, tree: int = TREE_BINARY, bypass_ms: int = 0,
                 route_kappa: float | None = None):
        o = ServerOpts()
        lib().tsqr_server_default_opts(ctypes.byref(o))
        o.hbm_budget, o.streams, o.max_inflight = hbm_budget, streams, max_inflight
        o.cache, o.prec, o.tree, o.bypass_ms = 1 if cache else 0, prec, tree, bypass_ms
        if route_kappa is not None:
            o.route_kappa = route_kappa
        h = ctypes.c_void_p()
        _check(lib().tsqr_server_create(ctypes.byref(o), ctypes.byref(h)), "tsqr_server_create")
        self._h = h
        self._keep = {}

    def submit(self, matrix_id: int, A: torch.Tensor, B: torch.Tensor, X: torch.Tensor,
               resid: torch.Tensor, info: torch.Tensor) -> int:
        m, n = A.shape
        k = 1 if B.dim() == 1 else B.shape[1]
        r = Request()
        r.matrix_id, r.m, r.n, r.k = matrix_id, m, n, k
        r.A = _host_colmajor_ptr(A, "A")
        r.B = _host_colmajor_ptr(B, "B")
        r.X = _host_colmajor_ptr(X, "X")
        r.resid = _host_colmajor_ptr(resid, "resid")
        r.info = _host_colmajor_ptr(info, "info")
        t = int(lib().tsqr_server_submit(self._h, ctypes.byref(r)))
        if t < 0:
            raise TSQRError(t, "tsqr_server_submit")
        self._keep[t] = (A, B, X, resid, info)
        return t

    def progress(self, wait: bool = False) -> int:
        rc = int(lib().tsqr_server_progress(self._h, 1 if wait else 0))
        if rc < 0:
            raise TSQRError(rc, "tsqr_server_progress")
        return rc

    def drain(self):
        while self.progress(wait=True) > 0:
            pass

    def status(self, t: int) -> int:
        return int(lib().tsqr_server_status(self._h, t))

    def times(self, t: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().tsqr_server_times(self._h, t, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "tsqr_server_times")
        return a.value, b.value, c.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().tsqr_server_get_stats(self._h, ctypes.byref(st)), "tsqr_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def release(self, t: int):
        """Drops the references kept for a finished request."""
        self._keep.pop(t, None)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tsqr_server_free(h)
            self._h = None
        self._keep = {}

    def __del__(self):
        self.close()


def server_now() -> float:
    return float(lib().tsqr_server_now())
