"""ctypes binding of libkmaa (include/km.h).

Argument marshalling only: tensors are checked for device, dtype and layout,
their data pointers and the current HIP stream are handed to the C ABI, and
status codes become exceptions.  All arithmetic runs in the library's HIP
kernels.  There is no fallback: if the library is missing or cannot be
loaded, every call raises.
"""

from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmaa.so")

KM_OK, KM_NOT_CONVERGED = 0, 1
KM_EINVAL, KM_ENOMEM, KM_EDEVICE, KM_EUNSUPPORTED, KM_ENONFINITE = -1, -2, -3, -4, -5
KM_X_F32, KM_X_BF16 = 0, 1
KM_GEMM_F32, KM_GEMM_BF16 = 0, 1
KM_FLAG_FIXED_M, KM_FLAG_LITERAL_RETURN, KM_FLAG_BOUNDS = 1, 2, 4
KM_TRACE_REC = 80


class KMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class _GStats(ct.Structure):
    _fields_ = [("changed", ct.c_int64), ("recheck_rows", ct.c_int64), ("near_tie_rows", ct.c_int64),
                ("empty_clusters", ct.c_int32), ("assign_ms", ct.c_float), ("update_ms", ct.c_float)]


class _Opts(ct.Structure):
    _fields_ = [("eps1", ct.c_double), ("eps2", ct.c_double), ("ridge", ct.c_double),
                ("m_init", ct.c_int32), ("max_iter", ct.c_int32), ("prec", ct.c_int),
                ("flags", ct.c_uint32), ("trace_C", ct.c_void_p), ("trace_rec", ct.c_void_p),
                ("m_traj", ct.c_void_p)]


class _SolveStats(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("accepted", ct.c_int32), ("rejected", ct.c_int32),
                ("assign_passes", ct.c_int32), ("m_final", ct.c_int32),
                ("assign_launches", ct.c_int32), ("recheck_rows", ct.c_int64),
                ("near_tie_rows", ct.c_int64), ("gemm_rows", ct.c_int64), ("bounds", ct.c_int32),
                ("device_ms", ct.c_double), ("assign_ms", ct.c_double)]


class _Job(ct.Structure):
    _fields_ = [("X", ct.c_void_p), ("xt", ct.c_int), ("N", ct.c_int64), ("d", ct.c_int32),
                ("K", ct.c_int32), ("C0", ct.c_void_p), ("C_out", ct.c_void_p), ("rho_out", ct.c_void_p),
                ("prec", ct.c_int)]


class _JobResult(ct.Structure):
    _fields_ = [("ticket", ct.c_int64), ("status", ct.c_int32), ("iters", ct.c_int32),
                ("E", ct.c_double), ("accepted", ct.c_int32), ("rejected", ct.c_int32),
                ("assign_passes", ct.c_int32), ("m_final", ct.c_int32),
                ("recheck_rows", ct.c_int64), ("near_tie_rows", ct.c_int64), ("latency_ms", ct.c_double)]


@dataclass
class JobResult:
    ticket: int
    status: int
    iters: int
    E: float
    accepted: int
    rejected: int
    assign_passes: int
    m_final: int
    recheck_rows: int
    near_tie_rows: int
    latency_ms: float


def _job_result(r: _JobResult) -> JobResult:
    return JobResult(r.ticket, r.status, r.iters, r.E, r.accepted, r.rejected, r.assign_passes,
                     r.m_final, r.recheck_rows, r.near_tie_rows, r.latency_ms)


@dataclass
class GStats:
    changed: int
    recheck_rows: int       # rows re-checked with float64 differences
    near_tie_rows: int      # float64 near ties (parity definition), all among the re-checked rows
    empty_clusters: int
    assign_ms: float = -1.0   # device times from HIP events when Context.set_timing(True)
    update_ms: float = -1.0


@dataclass
class SolveStats:
    iters: int
    accepted: int
    rejected: int
    assign_passes: int
    m_final: int
    recheck_rows: int
    near_tie_rows: int
    gemm_rows: int          # rows through the distance GEMM, all passes (N per pass without bounds)
    bounds: int             # 1 if row bounds were in use
    device_ms: float
    assign_ms: float
    assign_launches: int
    status: int
    m_traj: list | None = None   # m after the dynamic-m rule per iteration (entry 0: initial m)


_lib = None


def load_library(path: str | None = None):
    """Load libkmaa.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libkmaa.so not found at {path}; build it with "
                           "`python -m paper_1805_10638_amd.build`")
    lib = ct.CDLL(path)
    vp, i32, i64, dbl = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_double
    lib.km_create.argtypes = [ct.c_int, vp, ct.POINTER(vp)]
    lib.km_create.restype = ct.c_int
    lib.km_destroy.argtypes = [vp]
    lib.km_destroy.restype = None
    lib.km_set_stream.argtypes = [vp, vp]
    lib.km_set_stream.restype = ct.c_int
    lib.km_set_timing.argtypes = [vp, ct.c_int]
    lib.km_set_timing.restype = ct.c_int
    lib.km_set_tile_shape.argtypes = [vp, ct.c_int, ct.c_int, i32, i32, i32]
    lib.km_set_tile_shape.restype = ct.c_int
    lib.km_get_tile_shape.argtypes = [vp, ct.c_int, ct.c_int, i32, i32]
    lib.km_get_tile_shape.restype = ct.c_int
    lib.km_job_workspace_bytes.argtypes = [ct.POINTER(_Job), i32]
    lib.km_job_workspace_bytes.restype = i64
    lib.km_engine_create.argtypes = [vp, i32, dbl, ct.POINTER(_Opts), i64, i32, ct.POINTER(vp)]
    lib.km_engine_create.restype = ct.c_int
    lib.km_engine_destroy.argtypes = [vp]
    lib.km_engine_destroy.restype = None
    lib.km_engine_submit.argtypes = [vp, ct.POINTER(_Job), ct.POINTER(ct.c_int64)]
    lib.km_engine_submit.restype = ct.c_int
    lib.km_engine_step.argtypes = [vp, i32, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)]
    lib.km_engine_set_share.argtypes = [vp, dbl]
    lib.km_engine_set_share.restype = ct.c_int
    lib.km_engine_step.restype = ct.c_int
    lib.km_engine_poll.argtypes = [vp, ct.POINTER(_JobResult)]
    lib.km_engine_poll.restype = i32
    lib.kmeans_solve_batch.argtypes = [vp, ct.POINTER(_Job), i32, i32, dbl, ct.POINTER(_Opts),
                                       ct.POINTER(_JobResult)]
    lib.kmeans_solve_batch.restype = ct.c_int
    lib.km_status_str.argtypes = [ct.c_int]
    lib.km_status_str.restype = ct.c_char_p
    lib.km_last_error.argtypes = [vp]
    lib.km_last_error.restype = ct.c_char_p
    lib.km_version.argtypes = []
    lib.km_version.restype = ct.c_int
    lib.km_opts_default.argtypes = [ct.POINTER(_Opts)]
    lib.km_opts_default.restype = None
    lib.kmeans_g.argtypes = [vp, vp, ct.c_int, i64, i32, i32, vp, ct.c_int, vp, vp, vp,
                             ct.POINTER(dbl), ct.POINTER(_GStats)]
    lib.kmeans_g.restype = ct.c_int
    lib.kmeans_g_noalloc.argtypes = lib.kmeans_g.argtypes
    lib.kmeans_g_noalloc.restype = ct.c_int
    lib.kmeans_solve.argtypes = [vp, vp, ct.c_int, i64, i32, i32, vp, i32, dbl,
                                 ct.POINTER(_Opts), vp, vp, ct.POINTER(dbl), ct.POINTER(i32),
                                 ct.POINTER(_SolveStats)]
    lib.kmeans_solve.restype = ct.c_int
    _lib = lib
    return lib


class Context:
    """A libkmaa context bound to one device (workspace + stream)."""

    def __init__(self, device: int | None = None, tuned: bool = True):
        self.lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ct.c_void_p()
        st = self.lib.km_create(self.device, None, ct.byref(h))
        if st != KM_OK:
            raise KMError(st, "km_create failed: " + self.lib.km_status_str(st).decode())
        self.h = h
        self.tuned_entries = 0
        if tuned:  # tile shapes measured by the autotuner (tiles_gfx950.json), if present
            from . import autotune
            self.tuned_entries = autotune.apply_table(self, autotune.load_table())

    def close(self):
        if getattr(self, "h", None):
            self.lib.km_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.km_set_stream(self.h, ct.c_void_p(s))

    def set_timing(self, on: bool):
        self.lib.km_set_timing(self.h, 1 if on else 0)

    def set_tile_shape(self, prec: str, xtype: str, d: int, K: int, shape: int):
        """Assignment tile shape for calls whose (prec, X type, width, K bucket)
        match; 0 is the built-in default (see km_set_tile_shape)."""
        st = self.lib.km_set_tile_shape(self.h, _prec(prec), _xt_name(xtype), d, K, shape)
        self._check(st, "km_set_tile_shape")

    def tile_shape(self, prec: str, xtype: str, d: int, K: int) -> int:
        return self.lib.km_get_tile_shape(self.h, _prec(prec), _xt_name(xtype), d, K)

    def _check(self, st: int, what: str, allow=(KM_OK,)):
        if st in allow:
            return
        msg = self.lib.km_last_error(self.h).decode() or self.lib.km_status_str(st).decode()
        raise KMError(st, f"{what}: {msg}")


_ctx: dict[int, Context] = {}


def _context(device: int) -> Context:
    c = _ctx.get(device)
    if c is None:
        c = Context(device)
        _ctx[device] = c
    return c


def _xtype(X: torch.Tensor) -> int:
    if X.dtype == torch.float32:
        return KM_X_F32
    if X.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return KM_X_BF16
    raise TypeError(f"X must be float32 or bfloat16 (got {X.dtype})")


def _xt_name(x) -> int:
    if x in ("f32", "float32", KM_X_F32):
        return KM_X_F32
    if x in ("bf16", "bfloat16", KM_X_BF16):
        return KM_X_BF16
    raise ValueError(f"unknown X type {x!r}")


def _prec(p) -> int:
    if p in ("f32", "fp32", KM_GEMM_F32, None):
        return KM_GEMM_F32
    if p in ("bf16", KM_GEMM_BF16):
        return KM_GEMM_BF16
    raise ValueError(f"unknown precision {p!r}")


def _check_dev(t: torch.Tensor, name: str, device: int):
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def kmeans_g(X: torch.Tensor, C: torch.Tensor, prec="f32", rho_prev: torch.Tensor | None = None,
             ctx: Context | None = None, out: tuple | None = None):
    """One application of G (assignment then update).

    Returns (rho int32 [N], C_out float32 [K,d], E float (energy of C), GStats).
    ``out`` = (rho, C_out) writes into caller-owned tensors."""
    return _g_call("kmeans_g", X, C, prec, rho_prev, ctx, out)


def kmeans_g_noalloc(X: torch.Tensor, C: torch.Tensor, out: tuple, prec="f32",
                     rho_prev: torch.Tensor | None = None, ctx: Context | None = None):
    """kmeans_g whose scratch is the library's fixed device array (no device
    allocation in the call); ``out`` = (rho int32 [N], C_out float32 [K,d]) is
    required.  Returns (rho, C_out, E, GStats)."""
    return _g_call("kmeans_g_noalloc", X, C, prec, rho_prev, ctx, out)


def _g_call(name, X, C, prec, rho_prev, ctx, out):
    dev = X.device.index
    ctx = ctx or _context(dev)
    _check_dev(X, "X", dev)
    _check_dev(C, "C", dev)
    if C.dtype != torch.float32:
        raise TypeError("C must be float32")
    N, d = X.shape
    K = C.shape[0]
    if C.shape[1] != d:
        raise ValueError("C must be K x d")
    if out is None:
        rho = torch.empty(N, dtype=torch.int32, device=X.device)
        C_out = torch.empty_like(C)
    else:
        rho, C_out = out
        _check_dev(rho, "rho", dev)
        _check_dev(C_out, "C_out", dev)
        if rho.dtype != torch.int32 or rho.numel() != N:
            raise ValueError("rho must be int32 with N entries")
        if C_out.dtype != torch.float32 or C_out.shape != C.shape:
            raise ValueError("C_out must be float32 K x d")
    E = ct.c_double()
    gs = _GStats()
    if rho_prev is not None:
        _check_dev(rho_prev, "rho_prev", dev)
        if rho_prev.dtype != torch.int32:
            raise TypeError("rho_prev must be int32")
    ctx._bind_stream()
    st = getattr(ctx.lib, name)(ctx.h, ct.c_void_p(X.data_ptr()), _xtype(X), N, d, K,
                          ct.c_void_p(C.data_ptr()), _prec(prec),
                          ct.c_void_p(rho_prev.data_ptr()) if rho_prev is not None else None,
                          ct.c_void_p(rho.data_ptr()), ct.c_void_p(C_out.data_ptr()),
                          ct.byref(E), ct.byref(gs))
    ctx._check(st, name)
    return rho, C_out, E.value, GStats(gs.changed, gs.recheck_rows, gs.near_tie_rows, gs.empty_clusters,
                                       gs.assign_ms, gs.update_ms)


def kmeans_solve(X: torch.Tensor, C0: torch.Tensor, m_max: int = 10, tol: float = 1e-6,
                 max_iter: int = 500, eps1: float = 0.02, eps2: float = 0.5, m_init: int = 2,
                 prec="f32", fixed_m: bool = False, literal_return: bool = False,
                 ridge: float = 1e-10, trace: bool = False, ctx: Context | None = None,
                 out: tuple | None = None, m_traj: bool = False, bounds: bool = False):
    """Anderson-accelerated Lloyd K-Means (Algorithm 1).

    Returns (C float32 [K,d], rho int32 [N], E, iters, SolveStats) and, with
    ``trace=True``, a dict with the per-iteration candidates and records."""
    dev = X.device.index
    ctx = ctx or _context(dev)
    _check_dev(X, "X", dev)
    _check_dev(C0, "C0", dev)
    if C0.dtype != torch.float32:
        raise TypeError("C0 must be float32")
    N, d = X.shape
    K = C0.shape[0]
    if out is None:
        C = torch.empty_like(C0)
        rho = torch.empty(N, dtype=torch.int32, device=X.device)
    else:
        C, rho = out
    o = _Opts()
    ctx.lib.km_opts_default(ct.byref(o))
    o.eps1, o.eps2, o.ridge = eps1, eps2, ridge
    o.m_init, o.max_iter, o.prec = m_init, max_iter, _prec(prec)
    o.flags = (KM_FLAG_FIXED_M if fixed_m else 0) | (KM_FLAG_LITERAL_RETURN if literal_return else 0) | \
        (KM_FLAG_BOUNDS if bounds else 0)
    tr = None
    if trace:
        tr = {"C": torch.zeros((max_iter + 1, K, d), dtype=torch.float32, device=X.device),
              "rec": torch.zeros((max_iter + 1, KM_TRACE_REC), dtype=torch.float64, device=X.device)}
        o.trace_C = tr["C"].data_ptr()
        o.trace_rec = tr["rec"].data_ptr()
    mt = None
    if m_traj:
        mt = (ct.c_int32 * (max_iter + 1))()
        o.m_traj = ct.cast(mt, ct.c_void_p)
    E = ct.c_double()
    it = ct.c_int32()
    ss = _SolveStats()
    ctx._bind_stream()
    st = ctx.lib.kmeans_solve(ctx.h, ct.c_void_p(X.data_ptr()), _xtype(X), N, d, K,
                              ct.c_void_p(C0.data_ptr()), m_max, tol, ct.byref(o),
                              ct.c_void_p(C.data_ptr()), ct.c_void_p(rho.data_ptr()),
                              ct.byref(E), ct.byref(it), ct.byref(ss))
    ctx._check(st, "kmeans_solve", allow=(KM_OK, KM_NOT_CONVERGED))
    stats = SolveStats(ss.iters, ss.accepted, ss.rejected, ss.assign_passes, ss.m_final,
                       ss.recheck_rows, ss.near_tie_rows, ss.gemm_rows, ss.bounds, ss.device_ms, ss.assign_ms,
                       ss.assign_launches, st,
                       list(mt[:it.value + 1]) if mt is not None else None)
    if trace:
        return C, rho, E.value, it.value, stats, tr
    return C, rho, E.value, it.value, stats


# ---------------------------------------------------------------------------
# Many instances at once
# ---------------------------------------------------------------------------

def _solver_opts(lib, m_init, max_iter, prec, eps1, eps2, ridge, fixed_m, literal_return):
    o = _Opts()
    lib.km_opts_default(ct.byref(o))
    o.eps1, o.eps2, o.ridge = eps1, eps2, ridge
    o.m_init, o.max_iter, o.prec = m_init, max_iter, _prec(prec)
    o.flags = (KM_FLAG_FIXED_M if fixed_m else 0) | (KM_FLAG_LITERAL_RETURN if literal_return else 0)
    return o


def _make_job(X: torch.Tensor, C0: torch.Tensor, out, dev: int, prec):
    _check_dev(X, "X", dev)
    _check_dev(C0, "C0", dev)
    if C0.dtype != torch.float32:
        raise TypeError("C0 must be float32")
    N, d = X.shape
    K = C0.shape[0]
    if C0.shape[1] != d:
        raise ValueError("C0 must be K x d")
    if out is None:
        C = torch.empty_like(C0)
        rho = torch.empty(N, dtype=torch.int32, device=X.device)
    else:
        C, rho = out
    j = _Job(X.data_ptr(), _xtype(X), N, d, K, C0.data_ptr(), C.data_ptr(), rho.data_ptr(), _prec(prec))
    return j, (X, C0, C, rho)


def kmeans_solve_batch(problems, m_max: int = 10, tol: float = 1e-6, max_iter: int = 500,
                       m_init: int = 2, prec="f32", eps1: float = 0.02, eps2: float = 0.5,
                       ridge: float = 1e-10, fixed_m: bool = False, literal_return: bool = False,
                       ctx: "Context | None" = None):
    """Solve many instances together (kmeans_solve_batch in km.h).

    ``problems`` is a list of (X, C0) or (X, C0, prec) tuples on one device
    (``prec`` defaults to the argument).  Returns a list of (C, rho,
    JobResult) in the same order."""
    if not problems:
        return []
    dev = problems[0][0].device.index
    ctx = ctx or _context(dev)
    jobs = (_Job * len(problems))()
    keep = []
    for i, p in enumerate(problems):
        jobs[i], k = _make_job(p[0], p[1], None, dev, p[2] if len(p) > 2 else prec)
        keep.append(k)
    res = (_JobResult * len(problems))()
    o = _solver_opts(ctx.lib, m_init, max_iter, prec, eps1, eps2, ridge, fixed_m, literal_return)
    ctx._bind_stream()
    st = ctx.lib.kmeans_solve_batch(ctx.h, jobs, len(problems), m_max, tol, ct.byref(o), res)
    ctx._check(st, "kmeans_solve_batch")
    return [(k[2], k[3], _job_result(res[i])) for i, k in enumerate(keep)]


class Engine:
    """Continuous batching of clustering jobs (km_engine_* in km.h).

    ``submit`` queues a job (its tensors are kept alive until its result is
    taken); ``step`` admits what fits the HBM budget and advances every
    active job by one iteration; ``poll`` returns finished jobs as
    (ticket, C, rho, JobResult)."""

    def __init__(self, m_max: int = 10, tol: float = 1e-6, max_iter: int = 500, m_init: int = 2,
                 prec="f32", eps1: float = 0.02, eps2: float = 0.5, ridge: float = 1e-10,
                 hbm_budget: int = 0, graphs: bool = False, ctx: "Context | None" = None,
                 device: int | None = None):
        dev = torch.cuda.current_device() if device is None else device
        self.ctx = ctx or _context(dev)
        self.lib = self.ctx.lib
        self.device = dev
        o = _solver_opts(self.lib, m_init, max_iter, prec, eps1, eps2, ridge, False, False)
        self.prec = prec
        self.m_max = m_max
        h = ct.c_void_p()
        self.ctx._bind_stream()
        st = self.lib.km_engine_create(self.ctx.h, m_max, tol, ct.byref(o), hbm_budget,
                                       1 if graphs else 0, ct.byref(h))
        self.ctx._check(st, "km_engine_create")
        self.h = h
        self._jobs = {}

    def workspace_bytes(self, X: torch.Tensor, K: int, prec=None) -> int:
        N, d = X.shape
        j = _Job(0, _xtype(X), N, d, K, 0, 0, 0, _prec(prec or self.prec))
        return int(self.lib.km_job_workspace_bytes(ct.byref(j), self.m_max))

    def submit(self, X: torch.Tensor, C0: torch.Tensor, out=None, prec=None) -> int:
        """Queue a job; ``prec`` (GEMM precision) defaults to the engine's."""
        j, keep = _make_job(X, C0, out, self.device, prec or self.prec)
        t = ct.c_int64()
        self.ctx._bind_stream()
        st = self.lib.km_engine_submit(self.h, ct.byref(j), ct.byref(t))
        self.ctx._check(st, "km_engine_submit")
        self._jobs[t.value] = keep
        return t.value

    def step(self, wait: bool = True):
        """Admit, launch, collect (see km_engine_step); returns (active, queued, ready)."""
        a, q, r = ct.c_int32(), ct.c_int32(), ct.c_int32()
        st = self.lib.km_engine_step(self.h, 1 if wait else 0, ct.byref(a), ct.byref(q), ct.byref(r))
        self.ctx._check(st, "km_engine_step")
        return a.value, q.value, r.value

    def set_share(self, frac: float):
        """Fraction of the device's resident assignment workgroups to use."""
        self.ctx._check(self.lib.km_engine_set_share(self.h, frac), "km_engine_set_share")

    def poll(self):
        out = []
        r = _JobResult()
        while self.lib.km_engine_poll(self.h, ct.byref(r)):
            keep = self._jobs.pop(r.ticket)
            out.append((r.ticket, keep[2], keep[3], _job_result(r)))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.km_engine_destroy(self.h)
            self.h = None
            self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
