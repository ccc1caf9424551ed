"""Python binding of the gfx950 alternating Newton CD solver for l1-regularized CGGMs.

Argument marshalling only: every arithmetic step runs in the HIP kernels of
``libcggm.so`` (built from ``csrc/`` by ``build.py``).  PyTorch provides device
memory and the stream.  There is no CPU fallback: importing works without the
library, but every call raises if ``libcggm.so`` is missing.

Entry points mirror ``include/cggm.h``: :func:`cggm_solve`,
:func:`cggm_solve_path`, :func:`cggm_objective`,
:func:`cggm_objective_noalloc`, :func:`cggm_lambda_direction`,
:func:`cggm_gradient`, :func:`cggm_sigma_columns`, :func:`cggm_partition_graph`, the
request server :class:`Server` (``cggm_server_*``), plus
``cggm_status_string`` and the workspace-size queries.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcggm.so")

CGGM_OK, CGGM_MAXITER, CGGM_STALLED = 0, 1, 2
CGGM_PRECISION_FP64, CGGM_PRECISION_MIXED = 0, 1
CGGM_EINVAL, CGGM_ENOTPD, CGGM_ELINESEARCH, CGGM_ENOMEM, CGGM_EHIP = -1, -2, -3, -4, -5
CGGM_ECAPACITY = -6
CGGM_SWEEP_TILED, CGGM_SWEEP_SEQUENTIAL = 0, 1
CGGM_F64, CGGM_F32 = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_vp = ctypes.c_void_p


class TraceEntry(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int), ("ls_trials", ctypes.c_int),
                ("sweep_fallbacks", ctypes.c_int), ("sweep_split", ctypes.c_int),
                ("f", ctypes.c_double), ("subgrad_l1", ctypes.c_double),
                ("l1", ctypes.c_double), ("alpha", ctypes.c_double),
                ("m_Lambda", ctypes.c_int64), ("m_Theta", ctypes.c_int64),
                ("nnz_Lambda", ctypes.c_int64), ("nnz_Theta", ctypes.c_int64),
                ("t_end_ms", ctypes.c_double), ("ms_gradient", ctypes.c_double),
                ("ms_lambda_cd", ctypes.c_double), ("ms_line_search", ctypes.c_double),
                ("ms_theta_cd", ctypes.c_double), ("delta", ctypes.c_double)]


class KernelStats(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int64 * 2), ("tiles", ctypes.c_int64 * 2),
                ("ms", (ctypes.c_double * 3) * 2), ("bytes", (ctypes.c_double * 3) * 2),
                ("flops", (ctypes.c_double * 3) * 2)]


STAGES = ("snapshot", "gauss_seidel", "update")


class Options(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("max_ls", ctypes.c_int),
                ("ls_beta", ctypes.c_double), ("ls_sigma", ctypes.c_double),
                ("stall_iters", ctypes.c_int), ("sweep", ctypes.c_int),
                ("tile", ctypes.c_int), ("lambda_passes", ctypes.c_int),
                ("precision", ctypes.c_int), ("mixed_min_q", ctypes.c_int),
                ("workspace_budget", ctypes.c_size_t),
                ("warm_Lambda", _vp), ("warm_Theta", _vp),
                ("trace", ctypes.POINTER(TraceEntry)), ("trace_cap", ctypes.c_int),
                ("trace_len", ctypes.c_int), ("kstats", ctypes.POINTER(KernelStats)),
                ("theta_passes", ctypes.c_int), ("split_level", ctypes.c_int),
                ("split_adapt", ctypes.c_int), ("blockwise", ctypes.c_int),
                ("sxx_cache_bytes", ctypes.c_size_t), ("graphs", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("X", _vp), ("Y", _vp), ("n", _i64), ("p", _i64), ("q", _i64),
                ("npath", ctypes.c_int), ("lamL", _dp), ("lamT", _dp), ("tol", ctypes.c_double),
                ("precision", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("lambda_passes", ctypes.c_int), ("mixed_min_q", ctypes.c_int),
                ("Lambda_out", _vp), ("Theta_out", _vp), ("dtype", ctypes.c_int),
                ("tile", ctypes.c_int)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("slot", ctypes.c_int), ("iters_total", ctypes.c_int),
                ("_pad", ctypes.c_int), ("t_submit_ms", ctypes.c_double),
                ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("footprint", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("max_running", ctypes.c_int),
                ("_pad", ctypes.c_int), ("pool_bytes", ctypes.c_size_t),
                ("peak_bytes_in_use", ctypes.c_size_t)]


PRECISIONS = {"fp64": CGGM_PRECISION_FP64, "mixed": CGGM_PRECISION_MIXED}


class CggmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> ctypes.CDLL:
    """Load libcggm.so; raises when it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1509_04681_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    lib.cggm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.cggm_default_options.restype = None
    lib.cggm_solve_workspace_bytes.argtypes = [_i64, _i64, _i64]
    lib.cggm_solve_workspace_bytes.restype = ctypes.c_size_t
    lib.cggm_solve.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double,
                               ctypes.c_double, ctypes.POINTER(Options), ctypes.POINTER(_vp), _vp]
    lib.cggm_solve.restype = ctypes.c_int
    lib.cggm_workspace_bytes.argtypes = [_i64, _i64, _i64, ctypes.POINTER(Options)]
    lib.cggm_workspace_bytes.restype = ctypes.c_size_t
    lib.cggm_solve_path.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, _dp,
                                    _dp,
                                    ctypes.c_double, ctypes.POINTER(Options), ctypes.POINTER(_vp),
                                    _vp]
    lib.cggm_solve_path.restype = ctypes.c_int
    lib.cggm_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int,
                                       ctypes.POINTER(_vp)]
    lib.cggm_server_create.restype = ctypes.c_int
    lib.cggm_server_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(_i64)]
    lib.cggm_server_submit.restype = ctypes.c_int
    lib.cggm_server_wait.argtypes = [_vp, _i64, ctypes.POINTER(RequestInfo), _dp,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.cggm_server_wait.restype = ctypes.c_int
    lib.cggm_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    lib.cggm_server_stats_get.restype = ctypes.c_int
    lib.cggm_server_destroy.argtypes = [_vp]
    lib.cggm_server_destroy.restype = None
    lib.cggm_result_info.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                     ctypes.POINTER(ctypes.c_int), _dp,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.cggm_result_info.restype = ctypes.c_int
    lib.cggm_result_copy.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int]
    lib.cggm_result_copy.restype = ctypes.c_int
    lib.cggm_result_dense.argtypes = [_vp, _vp, _vp, ctypes.c_int]
    lib.cggm_result_dense.restype = ctypes.c_int
    lib.cggm_result_free.argtypes = [_vp]
    lib.cggm_result_free.restype = None
    lib.cggm_objective.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _vp, _vp,
                                   ctypes.c_double, ctypes.c_double, _dp, _vp]
    lib.cggm_objective.restype = ctypes.c_int
    lib.cggm_objective_noalloc.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _vp, _vp,
                                           ctypes.c_double, ctypes.c_double, _dp, _vp]
    lib.cggm_objective_noalloc.restype = ctypes.c_int
    lib.cggm_autotune_tile.argtypes = [_i64, _i64, _i64, ctypes.POINTER(Options), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int), _dp, _vp]
    lib.cggm_autotune_tile.restype = ctypes.c_int
    lib.cggm_lambda_direction.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _vp, _vp,
                                          ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(Options), _vp, _vp, _vp, _vp]
    lib.cggm_lambda_direction.restype = ctypes.c_int
    lib.cggm_gradient.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int, _vp, _vp, _vp, _vp,
                                  _vp]
    lib.cggm_gradient.restype = ctypes.c_int
    lib.cggm_sigma_columns.argtypes = [_vp, _vp, _vp, _i64, _vp, _i64, ctypes.c_double,
                                       ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double), _vp]
    lib.cggm_sigma_columns.restype = ctypes.c_int
    lib.cggm_partition_graph.argtypes = [_i64, _vp, _vp, _i64, ctypes.c_double, _vp,
                                         ctypes.POINTER(_i64)]
    lib.cggm_partition_graph.restype = ctypes.c_int
    lib.cggm_status_string.argtypes = [ctypes.c_int]
    lib.cggm_status_string.restype = ctypes.c_char_p
    lib.cggm_last_error.argtypes = []
    lib.cggm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def cggm_status_string(code: int) -> str:
    return load().cggm_status_string(code).decode()


def _check(code: int, allow_warning: bool = True) -> int:
    if code < 0 or (code > 0 and not allow_warning):
        lib = load()
        raise CggmError(code, f"{lib.cggm_status_string(code).decode()}: "
                              f"{lib.cggm_last_error().decode()}")
    return code


def _dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a GPU device")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    return ctypes.c_void_p(t.data_ptr())


def _inputs(X, Y):
    """Device pointers of X and Y and their element type (both float64 or both
    float32)."""
    import torch
    for t, name in ((X, "X"), (Y, "Y")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a torch tensor on a GPU device")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous (row-major)")
    types = {torch.float64: CGGM_F64, torch.float32: CGGM_F32}
    if X.dtype not in types or X.dtype != Y.dtype:
        raise TypeError("X and Y must both be float64 or both float32")
    return ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), types[X.dtype]


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


@dataclasses.dataclass
class SolveResult:
    Lambda: "torch.Tensor"        # dense q x q (device)
    Theta: "torch.Tensor"         # dense p x q (device)
    f: float
    iters: int
    status: int
    nnz_Lambda: int
    nnz_Theta: int
    trace: list
    # CD sweep kernel statistics when cggm_solve(..., kernel_stats=True):
    # {"<lambda|theta>_<snapshot|gauss_seidel|update>": {launches, tiles, ms, bytes, flops}}
    kernel_stats: dict | None = None
    # host CSR ((rowptr, col, val) of Lambda (full symmetric), same of Theta)
    # when cggm_solve(..., keep_csr=True)
    csr: tuple | None = None


def _options(lib, *, max_iter, max_ls, ls_beta, ls_sigma, stall_iters, sweep, tile,
             lambda_passes, precision, workspace_budget, warm_Lambda, warm_Theta,
             mixed_min_q=None, theta_passes=1, split_level=0, split_adapt=True,
             blockwise=False, sxx_cache_bytes=0, graphs=False) -> Options:
    opt = Options()
    lib.cggm_default_options(ctypes.byref(opt))
    opt.max_iter, opt.max_ls, opt.ls_beta, opt.ls_sigma = max_iter, max_ls, ls_beta, ls_sigma
    opt.stall_iters, opt.sweep, opt.tile = stall_iters, sweep, tile
    opt.lambda_passes, opt.theta_passes = lambda_passes, theta_passes
    opt.split_level, opt.split_adapt = split_level, int(bool(split_adapt))
    opt.blockwise, opt.sxx_cache_bytes = int(bool(blockwise)), int(sxx_cache_bytes)
    opt.graphs = int(bool(graphs))
    opt.precision = PRECISIONS[precision]
    if mixed_min_q is not None:
        opt.mixed_min_q = mixed_min_q
    opt.workspace_budget = workspace_budget
    if warm_Lambda is not None:
        opt.warm_Lambda = _dev(warm_Lambda, "warm_Lambda").value
    if warm_Theta is not None:
        opt.warm_Theta = _dev(warm_Theta, "warm_Theta").value
    return opt


def _take_result(lib, res, p, q, device, keep_csr):
    """Copy a result handle out (dense device tensors, optional host CSR) and free it."""
    import torch
    try:
        nL, nT, it, f, st = _i64(), _i64(), ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        _check(lib.cggm_result_info(res, ctypes.byref(nL), ctypes.byref(nT), ctypes.byref(it),
                                    ctypes.byref(f), ctypes.byref(st)))
        Lam = torch.empty((q, q), dtype=torch.float64, device=device)
        Th = torch.empty((p, q), dtype=torch.float64, device=device)
        _check(lib.cggm_result_dense(res, ctypes.c_void_p(Lam.data_ptr()),
                                     ctypes.c_void_p(Th.data_ptr()), 0))
        csr = None
        if keep_csr:
            Lr, Lc, Lv = (np.empty(q + 1, np.int64), np.empty(max(nL.value, 1), np.int32),
                          np.empty(max(nL.value, 1), np.float64))
            Tr, Tc, Tv = (np.empty(p + 1, np.int64), np.empty(max(nT.value, 1), np.int32),
                          np.empty(max(nT.value, 1), np.float64))
            _check(lib.cggm_result_copy(res, *(ctypes.c_void_p(a.ctypes.data)
                                               for a in (Lr, Lc, Lv, Tr, Tc, Tv)), 1))
            csr = ((Lr, Lc[:nL.value], Lv[:nL.value]), (Tr, Tc[:nT.value], Tv[:nT.value]))
    finally:
        lib.cggm_result_free(res)
    return SolveResult(Lambda=Lam, Theta=Th, f=f.value, iters=it.value, status=st.value,
                       nnz_Lambda=nL.value, nnz_Theta=nT.value, trace=[], csr=csr)


def _trace_list(trace_buf, n):
    return [{k: getattr(trace_buf[i], k) for k, _ in TraceEntry._fields_ if k != "_pad"}
            for i in range(n)]


def cggm_solve(X, Y, lam_Lambda: float, lam_Theta: float, tol: float = 1e-2, *,
               max_iter: int = 500, max_ls: int = 30, ls_beta: float = 0.5,
               ls_sigma: float = 1e-3, stall_iters: int = 3, sweep: int = CGGM_SWEEP_TILED,
               tile: int = 0, lambda_passes: int = 0, precision: str = "fp64",
               mixed_min_q: int | None = None, workspace_budget: int = 0,
               warm_Lambda=None, warm_Theta=None, trace_cap: int | None = None,
               keep_csr: bool = False, kernel_stats: bool = False,
               theta_passes: int = 1, split_level: int = 0, split_adapt: bool = True,
               blockwise: bool = False, sxx_cache_bytes: int = 0, graphs: bool = False,
               stream=None) -> SolveResult:
    """Alternating Newton CD (Algorithm 1) on device X (n x p) and Y (n x q), float64."""
    lib = load()
    n, p = X.shape
    q = Y.shape[1]
    opt = _options(lib, max_iter=max_iter, max_ls=max_ls, ls_beta=ls_beta, ls_sigma=ls_sigma,
                   stall_iters=stall_iters, sweep=sweep, tile=tile,
                   lambda_passes=lambda_passes, precision=precision,
                   workspace_budget=workspace_budget, warm_Lambda=warm_Lambda,
                   warm_Theta=warm_Theta, mixed_min_q=mixed_min_q,
                   theta_passes=theta_passes, split_level=split_level,
                   split_adapt=split_adapt, blockwise=blockwise,
                   sxx_cache_bytes=sxx_cache_bytes, graphs=graphs)
    cap = (max_iter + 1) if trace_cap is None else trace_cap
    trace_buf = (TraceEntry * max(cap, 1))()
    opt.trace = ctypes.cast(trace_buf, ctypes.POINTER(TraceEntry)) if cap > 0 else None
    opt.trace_cap = cap
    ks = KernelStats() if kernel_stats else None
    if ks is not None:
        opt.kstats = ctypes.pointer(ks)
    res = ctypes.c_void_p()
    Xp, Yp, dtype = _inputs(X, Y)
    code = lib.cggm_solve(Xp, Yp, n, p, q, dtype, float(lam_Lambda),
                          float(lam_Theta), float(tol), ctypes.byref(opt), ctypes.byref(res),
                          _stream(stream))
    if not (code == CGGM_ELINESEARCH and res.value):    # that status still returns a result
        _check(code)
    out = _take_result(lib, res, p, q, X.device, keep_csr)
    out.trace = _trace_list(trace_buf, opt.trace_len)
    if ks is not None:
        kst = {}
        for k, sw in enumerate(("lambda", "theta")):
            for j, stage in enumerate(STAGES):
                kst[f"{sw}_{stage}"] = {"launches": ks.waves[k], "tiles": ks.tiles[k],
                                        "ms": ks.ms[k][j], "bytes": ks.bytes[k][j],
                                        "flops": ks.flops[k][j]}
        out.kernel_stats = kst
    return out


def cggm_solve_path(X, Y, lam_Lambda, lam_Theta, tol: float = 1e-2, *,
                    max_iter: int = 500, max_ls: int = 30, ls_beta: float = 0.5,
                    ls_sigma: float = 1e-3, stall_iters: int = 3,
                    sweep: int = CGGM_SWEEP_TILED, tile: int = 0, lambda_passes: int = 0,
                    precision: str = "fp64", mixed_min_q: int | None = None,
                    workspace_budget: int = 0, warm_Lambda=None,
                    warm_Theta=None, trace_cap: int | None = None, keep_csr: bool = False,
                    theta_passes: int = 1, split_level: int = 0, split_adapt: bool = True,
                    blockwise: bool = False, sxx_cache_bytes: int = 0, graphs: bool = False,
                    stream=None) -> list:
    """Warm-started regularisation path: one SolveResult per (lam_Lambda[k], lam_Theta[k])."""
    lib = load()
    n, p = X.shape
    q = Y.shape[1]
    lamL = np.ascontiguousarray(lam_Lambda, dtype=np.float64).ravel()
    lamT = np.ascontiguousarray(lam_Theta, dtype=np.float64).ravel()
    if lamL.size != lamT.size or lamL.size < 1:
        raise ValueError("lam_Lambda and lam_Theta must have the same length >= 1")
    npath = lamL.size
    opt = _options(lib, max_iter=max_iter, max_ls=max_ls, ls_beta=ls_beta, ls_sigma=ls_sigma,
                   stall_iters=stall_iters, sweep=sweep, tile=tile,
                   lambda_passes=lambda_passes, precision=precision,
                   workspace_budget=workspace_budget, warm_Lambda=warm_Lambda,
                   warm_Theta=warm_Theta, mixed_min_q=mixed_min_q,
                   theta_passes=theta_passes, split_level=split_level,
                   split_adapt=split_adapt, blockwise=blockwise,
                   sxx_cache_bytes=sxx_cache_bytes, graphs=graphs)
    cap = npath * (max_iter + 1) if trace_cap is None else trace_cap
    trace_buf = (TraceEntry * max(cap, 1))()
    opt.trace = ctypes.cast(trace_buf, ctypes.POINTER(TraceEntry)) if cap > 0 else None
    opt.trace_cap = cap
    res = (ctypes.c_void_p * npath)()
    Xp, Yp, dtype = _inputs(X, Y)
    code = lib.cggm_solve_path(Xp, Yp, n, p, q, dtype, npath,
                               lamL.ctypes.data_as(_dp), lamT.ctypes.data_as(_dp), float(tol),
                               ctypes.byref(opt), res, _stream(stream))
    if not (code == CGGM_ELINESEARCH and res[0]):
        _check(code)
    outs = [_take_result(lib, ctypes.c_void_p(res[k]), p, q, X.device, keep_csr)
            for k in range(npath)]
    trace = _trace_list(trace_buf, opt.trace_len)
    k = -1
    for rec in trace:                       # records of point k start at iter 0
        if rec["iter"] == 0:
            k += 1
        if 0 <= k < npath:
            outs[k].trace.append(rec)
    return outs


def cggm_objective(X, Y, Lambda, Theta, lam_Lambda: float, lam_Theta: float,
                   stream=None) -> float:
    """f(Lambda, Theta) of Eq. (1); raises CggmError(CGGM_ENOTPD) when Lambda is not PD."""
    lib = load()
    n, p = X.shape
    q = Y.shape[1]
    f = ctypes.c_double()
    Xp, Yp, dtype = _inputs(X, Y)
    _check(lib.cggm_objective(Xp, Yp, n, p, q, dtype, _dev(Lambda, "Lambda"),
                              _dev(Theta, "Theta"), float(lam_Lambda), float(lam_Theta),
                              ctypes.byref(f), _stream(stream)))
    return f.value


def cggm_objective_noalloc(X, Y, Lambda, Theta, lam_Lambda: float, lam_Theta: float,
                           stream=None) -> float:
    """cggm_objective from the library's static device scratch (no device
    allocation); raises CggmError(CGGM_ECAPACITY) for shapes whose workspace
    exceeds it."""
    lib = load()
    n, p = X.shape
    q = Y.shape[1]
    f = ctypes.c_double()
    Xp, Yp, dtype = _inputs(X, Y)
    _check(lib.cggm_objective_noalloc(Xp, Yp, n, p, q, dtype,
                                      _dev(Lambda, "Lambda"), _dev(Theta, "Theta"),
                                      float(lam_Lambda), float(lam_Theta), ctypes.byref(f),
                                      _stream(stream)))
    return f.value


def cggm_autotune_tile(n: int, p: int, q: int, precision: str = "fp64", iters: int = 2,
                       graphs: bool = False, stream=None):
    """(best tile edge, {edge: ms per iteration}) for problems of shape (n, p, q)."""
    lib = load()
    opt = Options()
    lib.cggm_default_options(ctypes.byref(opt))
    opt.precision = PRECISIONS[precision]
    opt.graphs = int(bool(graphs))
    tile = ctypes.c_int()
    ms = (ctypes.c_double * 3)()
    _check(lib.cggm_autotune_tile(n, p, q, ctypes.byref(opt), int(iters), ctypes.byref(tile),
                                  ms, _stream(stream)))
    return tile.value, {16: ms[0], 32: ms[1], 64: ms[2]}


def cggm_lambda_direction(X, Y, Lambda, Theta, lam_Lambda: float, lam_Theta: float, *,
                          lambda_passes: int = 0, sweep: int = CGGM_SWEEP_TILED, tile: int = 0,
                          precision: str = "fp64", mixed_min_q: int | None = None,
                          split_level: int = 0, stream=None):
    """(D, U, V): one Lambda Newton direction at (Lambda, Theta), the maintained
    U = D Sigma and V = Theta Sigma as the solver forms them (device tensors)."""
    import torch
    lib = load()
    n, p = X.shape
    q = Y.shape[1]
    opt = _options(lib, max_iter=1, max_ls=30, ls_beta=0.5, ls_sigma=1e-3, stall_iters=0,
                   sweep=sweep, tile=tile, lambda_passes=lambda_passes, precision=precision,
                   workspace_budget=0, warm_Lambda=None, warm_Theta=None,
                   mixed_min_q=mixed_min_q, split_level=split_level)
    D = torch.empty((q, q), dtype=torch.float64, device=X.device)
    U = torch.empty((q, q), dtype=torch.float64, device=X.device)
    V = torch.empty((p, q), dtype=torch.float64, device=X.device)
    Xp, Yp, dtype = _inputs(X, Y)
    _check(lib.cggm_lambda_direction(Xp, Yp, n, p, q, dtype, _dev(Lambda, "Lambda"),
                                     _dev(Theta, "Theta"), float(lam_Lambda), float(lam_Theta),
                                     ctypes.byref(opt), _dev(D, "D"), _dev(U, "U"), _dev(V, "V"),
                                     _stream(stream)))
    return D, U, V


def cggm_gradient(X, Y, Lambda, Theta, stream=None):
    """(G_Lambda, G_Theta) of Eq. (3) as new device tensors."""
    import torch
    lib = load()
    n, p = X.shape
    q = Y.shape[1]
    GL = torch.empty((q, q), dtype=torch.float64, device=X.device)
    GT = torch.empty((p, q), dtype=torch.float64, device=X.device)
    Xp, Yp, dtype = _inputs(X, Y)
    _check(lib.cggm_gradient(Xp, Yp, n, p, q, dtype, _dev(Lambda, "Lambda"),
                             _dev(Theta, "Theta"), _dev(GL, "G_Lambda"), _dev(GT, "G_Theta"),
                             _stream(stream)))
    return GL, GT


@dataclasses.dataclass
class SigmaColumns:
    Sigma_C: object        # q x k device tensor: column t is Sigma's column cols[t]
    iters: int             # the most iterations a batch of 64 columns ran
    resid: float           # largest final residual norm over the columns
    status: int            # CGGM_OK, or CGGM_MAXITER when some column missed tol


def cggm_sigma_columns(rowptr, col, val, cols, tol=1e-12, max_iter=1000, stream=None):
    """Columns `cols` of Sigma = Lambda^{-1} by conjugate gradients on a sparse
    symmetric positive definite Lambda (Sec. 4.1): Lambda in CSR as device
    tensors (rowptr int64 of q + 1 entries, col int32 and val float64 of
    rowptr[q] entries, both triangles stored); `cols` a sequence of column
    indices.  Raises CggmError on an error status."""
    import torch
    lib = load()
    for t, name, dt in ((rowptr, "rowptr", torch.int64), (col, "col", torch.int32),
                        (val, "val", torch.float64)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a torch tensor on a GPU device")
        if t.dtype != dt or t.dim() != 1 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous 1-D {dt} tensor")
    q = rowptr.numel() - 1
    if q < 1:
        raise ValueError("rowptr must hold q + 1 >= 2 offsets")
    nnz = int(rowptr[-1].item())
    if col.numel() != nnz or val.numel() != nnz:
        raise ValueError(f"col and val must hold rowptr[q] = {nnz} entries")
    cidx = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    if cidx.ndim != 1 or (cidx.size and (cidx.min() < 0 or cidx.max() >= q)):
        raise ValueError("cols must be a 1-D sequence of indices in [0, q)")
    cidx = cidx.astype(np.int32)
    k = int(cidx.size)
    out = torch.empty((q, max(k, 1)), dtype=torch.float64, device=rowptr.device)[:, :k]
    it, res = ctypes.c_int(0), ctypes.c_double(0.0)
    st = _check(lib.cggm_sigma_columns(
        ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(col.data_ptr()),
        ctypes.c_void_p(val.data_ptr()), q, cidx.ctypes.data_as(ctypes.c_void_p), k, tol,
        max_iter, ctypes.c_void_p(out.data_ptr()), ctypes.byref(it), ctypes.byref(res),
        _stream(stream)))
    return SigmaColumns(out, int(it.value), float(res.value), st)


def cggm_partition_graph(rowptr, col, nparts: int, imbalance: float = 0.05):
    """Balanced partition of a graph into `nparts` parts with few cut edges
    (the block-wise method's graph clustering, Sec. 4.1 and 4.2), computed on
    the host: `rowptr` (n + 1) and `col` (rowptr[n]) are the adjacency
    pattern in CSR as host arrays, taken as undirected.  Returns (part of
    each vertex as an int32 array, number of cut edges)."""
    lib = load()
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.size - 1
    if n < 1 or cl.size != int(rp[-1]):
        raise ValueError("rowptr must hold n + 1 >= 2 offsets and col rowptr[n] entries")
    part = np.empty(n, dtype=np.int32)
    cut = _i64(0)
    _check(lib.cggm_partition_graph(n, rp.ctypes.data_as(_vp), cl.ctypes.data_as(_vp), nparts,
                                    imbalance, part.ctypes.data_as(_vp), ctypes.byref(cut)))
    return part, int(cut.value)


def cggm_solve_workspace_bytes(n: int, p: int, q: int) -> int:
    return int(load().cggm_solve_workspace_bytes(n, p, q))


def cggm_workspace_bytes(n: int, p: int, q: int, precision: str = "fp64",
                         blockwise: bool = False, sxx_cache_bytes: int = 0) -> int:
    lib = load()
    opt = Options()
    lib.cggm_default_options(ctypes.byref(opt))
    opt.precision = PRECISIONS[precision]
    opt.blockwise, opt.sxx_cache_bytes = int(bool(blockwise)), int(sxx_cache_bytes)
    return int(lib.cggm_workspace_bytes(n, p, q, ctypes.byref(opt)))


class Server:
    """Continuous-batching request server (``cggm_server_*``): regularisation
    paths of independent problems solved concurrently on the current device,
    admitted as worker slots and pool memory free up."""

    def __init__(self, slots: int = 4, pool_bytes: int | None = None, max_bypass: int = 8):
        import torch
        self._lib = load()
        if pool_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            pool_bytes = int(free * 0.5)
        h = ctypes.c_void_p()
        _check(self._lib.cggm_server_create(int(slots), int(pool_bytes), int(max_bypass),
                                            ctypes.byref(h)))
        self._h = h
        self._held = {}         # ticket -> objects the device work reads or writes

    def submit(self, X, Y, lam_Lambda, lam_Theta, tol: float = 1e-2, *,
               precision: str = "fp64", max_iter: int = 0, lambda_passes: int = 0,
               mixed_min_q: int | None = None, Lambda_out=None, Theta_out=None,
               tile: int = 0) -> int:
        n, p = X.shape
        q = Y.shape[1]
        lamL = np.ascontiguousarray(lam_Lambda, dtype=np.float64).ravel()
        lamT = np.ascontiguousarray(lam_Theta, dtype=np.float64).ravel()
        if lamL.size != lamT.size:
            raise ValueError("lam_Lambda and lam_Theta must have the same length")
        npath = lamL.size
        r = Request()
        Xp, Yp, r.dtype = _inputs(X, Y)
        r.X, r.Y = Xp.value, Yp.value
        r.n, r.p, r.q, r.npath = n, p, q, npath
        r.lamL, r.lamT = lamL.ctypes.data_as(_dp), lamT.ctypes.data_as(_dp)
        r.tol, r.precision = float(tol), PRECISIONS[precision]
        r.max_iter, r.lambda_passes = int(max_iter), int(lambda_passes)
        r.mixed_min_q = -1 if mixed_min_q is None else int(mixed_min_q)
        r.tile = int(tile)
        for t, name, shape in ((Lambda_out, "Lambda_out", (npath, q, q)),
                               (Theta_out, "Theta_out", (npath, p, q))):
            if t is not None and tuple(t.shape) != shape:
                raise ValueError(f"{name} must have shape {shape}")
        r.Lambda_out = _dev(Lambda_out, "Lambda_out").value if Lambda_out is not None else None
        r.Theta_out = _dev(Theta_out, "Theta_out").value if Theta_out is not None else None
        ticket = _i64()
        _check(self._lib.cggm_server_submit(self._h, ctypes.byref(r), ctypes.byref(ticket)))
        self._held[ticket.value] = (X, Y, Lambda_out, Theta_out, npath)
        return ticket.value

    def wait(self, ticket: int) -> dict:
        npath = self._held[ticket][4]
        info = RequestInfo()
        f = np.zeros(npath, np.float64)
        it = np.zeros(npath, np.int32)
        code = self._lib.cggm_server_wait(self._h, int(ticket), ctypes.byref(info),
                                          f.ctypes.data_as(_dp),
                                          it.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        self._held.pop(ticket, None)
        if code != CGGM_ELINESEARCH:
            _check(code)
        return {"status": info.status, "slot": info.slot, "iters_total": info.iters_total,
                "t_submit_ms": info.t_submit_ms, "t_admit_ms": info.t_admit_ms,
                "t_done_ms": info.t_done_ms, "footprint": int(info.footprint),
                "f": f.tolist(), "iters": it.tolist()}

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.cggm_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "_pad"}

    def close(self):
        if self._h is not None and self._h.value:
            self._lib.cggm_server_destroy(self._h)
        self._h = None
        self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
