"""Plain FP64 CPU oracle for alternating Newton coordinate descent (ANCD).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg import this package; the GPU library never does,
and nothing here is shared with it.  The arithmetic lives in ``cggm_oracle.c``
(plain loops, sequential Gauss-Seidel coordinate descent, its own Cholesky);
this module only compiles it with gcc and marshals numpy arrays through ctypes.

Each function names the part of the paper (McCarter & Kim, AISTATS 2016) it
follows; see the C source for the readings taken where the paper is garbled.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cggm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcggm_oracle.so")
_lock = threading.Lock()
_lib = None

ORC_OK, ORC_MAXITER, ORC_STALLED, ORC_NOTPD = 0, 1, 2, -2

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)
_i64 = ctypes.c_int64
_d = ctypes.c_double


class _Trace(ctypes.Structure):
    _fields_ = [("f", _dp), ("subgrad", _dp), ("l1", _dp), ("alpha", _dp),
                ("mL", _i64p), ("mT", _i64p), ("nnzL", _i64p), ("nnzT", _i64p),
                ("ls_trials", _ip)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/libcggm_oracle.so."""
    with _lock:
        if force or not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            tmp = _LIB_PATH + f".tmp{os.getpid()}"
            cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
                   "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True, cwd=_HERE)
            os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_stats.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp, _dp]
    lib.orc_stats.restype = None
    lib.orc_cholesky.argtypes = [_i64, _dp, _dp]
    lib.orc_cholesky.restype = ctypes.c_int
    lib.orc_inverse_from_cholesky.argtypes = [_i64, _dp, _dp]
    lib.orc_inverse_from_cholesky.restype = None
    lib.orc_objective.argtypes = [_i64, _i64, _dp, _dp, _dp, _dp, _dp, _d, _d, _dp]
    lib.orc_objective.restype = ctypes.c_int
    lib.orc_gradient.argtypes = [_i64, _i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_gradient.restype = ctypes.c_int
    lib.orc_active_sets.argtypes = [_i64, _i64, _dp, _dp, _dp, _dp, _d, _d, _u8p, _u8p]
    lib.orc_active_sets.restype = None
    lib.orc_lambda_direction.argtypes = [_i64, _dp, _dp, _dp, _dp, _u8p, _d, ctypes.c_int,
                                         _dp]
    lib.orc_lambda_direction.restype = None
    lib.orc_line_search.argtypes = [_i64, _i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _d, _d,
                                    _d, _d, _d, ctypes.c_int, _dp, _dp, _ip]
    lib.orc_line_search.restype = ctypes.c_int
    lib.orc_theta_sweep.argtypes = [_i64, _i64, _dp, _dp, _dp, _u8p, _d, _dp]
    lib.orc_theta_sweep.restype = None
    lib.orc_solve.argtypes = [_i64, _i64, _i64, _dp, _dp, _d, _d, _d, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _ip, _dp,
                              ctypes.POINTER(_Trace)]
    lib.orc_solve.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    if a.dtype == np.uint8:
        return a.ctypes.data_as(_u8p)
    return a.ctypes.data_as(_dp)


def stats(X, Y):
    """Sxx = X^T X/n, Sxy = X^T Y/n, Syy = Y^T Y/n, uncentred (Sec. 2.1)."""
    X, Y = _c(X), _c(Y)
    n, p = X.shape
    q = Y.shape[1]
    Sxx, Sxy, Syy = np.empty((p, p)), np.empty((p, q)), np.empty((q, q))
    _load().orc_stats(n, p, q, _p(X), _p(Y), _p(Sxx), _p(Sxy), _p(Syy))
    return Sxx, Sxy, Syy


def cholesky(A):
    """Lower Cholesky factor, or None when A is not positive definite."""
    A = _c(A)
    L = np.empty_like(A)
    rc = _load().orc_cholesky(A.shape[0], _p(A), _p(L))
    return L if rc == ORC_OK else None


def inverse(A):
    """Sigma = A^{-1} through the oracle's own Cholesky (None if not PD)."""
    L = cholesky(A)
    if L is None:
        return None
    S = np.empty_like(L)
    _load().orc_inverse_from_cholesky(L.shape[0], _p(L), _p(S))
    return S


def objective(S, Lambda, Theta, lamL, lamT):
    """f of Eq. (1) given S = (Sxx, Sxy, Syy); None when Lambda is not PD."""
    Sxx, Sxy, Syy = (_c(a) for a in S)
    Lambda, Theta = _c(Lambda), _c(Theta)
    p, q = Theta.shape
    f = ctypes.c_double()
    rc = _load().orc_objective(p, q, _p(Sxx), _p(Sxy), _p(Syy), _p(Lambda), _p(Theta),
                               lamL, lamT, ctypes.byref(f))
    return f.value if rc == ORC_OK else None


def gradient(S, Lambda, Theta):
    """(G_Lambda, G_Theta, Sigma, Psi) of Eq. (3); None when Lambda is not PD."""
    Sxx, Sxy, Syy = (_c(a) for a in S)
    Lambda, Theta = _c(Lambda), _c(Theta)
    p, q = Theta.shape
    GL, GT = np.empty((q, q)), np.empty((p, q))
    Sg, Ps = np.empty((q, q)), np.empty((q, q))
    rc = _load().orc_gradient(p, q, _p(Sxx), _p(Sxy), _p(Syy), _p(Lambda), _p(Theta),
                              _p(GL), _p(GT), _p(Sg), _p(Ps))
    return (GL, GT, Sg, Ps) if rc == ORC_OK else None


def active_sets(GL, GT, Lambda, Theta, lamL, lamT):
    """Byte masks of S_Lambda (upper triangle) and S_Theta (Sec. 2.2)."""
    GL, GT, Lambda, Theta = _c(GL), _c(GT), _c(Lambda), _c(Theta)
    p, q = GT.shape
    aL, aT = np.empty((q, q), np.uint8), np.empty((p, q), np.uint8)
    _load().orc_active_sets(p, q, _p(GL), _p(GT), _p(Lambda), _p(Theta), lamL, lamT,
                            _p(aL), _p(aT))
    return aL.astype(bool), aT.astype(bool)


def lambda_direction(Sigma, Psi, GL, Lambda, actL, lamL, passes=1):
    """Lexicographic CD passes (one by default, Sec. 3) for the Newton direction
    of Eq. (6), from D = 0."""
    Sigma, Psi, GL, Lambda = _c(Sigma), _c(Psi), _c(GL), _c(Lambda)
    actL = _c(actL, np.uint8)
    q = Sigma.shape[0]
    D = np.empty((q, q))
    _load().orc_lambda_direction(q, _p(Sigma), _p(Psi), _p(GL), _p(Lambda), _p(actL),
                                 lamL, int(passes), _p(D))
    return D


def line_search(S, Lambda, Theta, D, GL, lamL, lamT, f0, beta=0.5, sigma=1e-3, max_ls=30):
    """Armijo step on Lambda (Algorithm 1). Returns (Lambda_new, alpha, f_new, trials)."""
    Sxx, Sxy, Syy = (_c(a) for a in S)
    Lam = np.array(Lambda, dtype=np.float64, order="C", copy=True)
    Theta, D, GL = _c(Theta), _c(D), _c(GL)
    p, q = Theta.shape
    a, f, tr = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _load().orc_line_search(p, q, _p(Sxx), _p(Sxy), _p(Syy), _p(Lam), _p(Theta), _p(D),
                            _p(GL), lamL, lamT, f0, beta, sigma, max_ls, ctypes.byref(a),
                            ctypes.byref(f), ctypes.byref(tr))
    return Lam, a.value, f.value, tr.value


def theta_sweep(S, Sigma, actT, lamT, Theta):
    """One lexicographic CD pass on Eq. (7); returns the updated Theta."""
    Sxx, Sxy, _ = (_c(a) for a in S)
    Th = np.array(Theta, dtype=np.float64, order="C", copy=True)
    Sigma, actT = _c(Sigma), _c(actT, np.uint8)
    p, q = Th.shape
    _load().orc_theta_sweep(p, q, _p(Sxx), _p(Sxy), _p(Sigma), _p(actT), lamT, _p(Th))
    return Th


@dataclasses.dataclass
class SolveResult:
    Lambda: np.ndarray
    Theta: np.ndarray
    f: float
    iters: int
    status: int
    trace: dict


def solve(X, Y, lamL, lamT, tol=1e-2, max_iter=200, stall_iters=0, Lambda0=None,
          Theta0=None, lambda_passes=1) -> SolveResult:
    """Alternating Newton CD (Algorithm 1) to the stopping rule of Sec. 5.1 with tol."""
    X, Y = _c(X), _c(Y)
    n, p = X.shape
    q = Y.shape[1]
    warm = Lambda0 is not None
    Lam = _c(Lambda0).copy() if warm else np.empty((q, q))
    Th = (_c(Theta0).copy() if Theta0 is not None else np.zeros((p, q))) if warm \
        else np.empty((p, q))
    m = max_iter + 1
    arrs = dict(f=np.full(m, np.nan), subgrad=np.full(m, np.nan), l1=np.full(m, np.nan),
                alpha=np.full(m, np.nan), mL=np.zeros(m, np.int64), mT=np.zeros(m, np.int64),
                nnzL=np.zeros(m, np.int64), nnzT=np.zeros(m, np.int64),
                ls_trials=np.zeros(m, np.int32))
    tr = _Trace(**{k: v.ctypes.data_as(_ip if v.dtype == np.int32 else
                                        (_i64p if v.dtype == np.int64 else _dp))
                   for k, v in arrs.items()})
    iters, f = ctypes.c_int(), ctypes.c_double()
    if lambda_passes < 1:
        raise ValueError("lambda_passes must be >= 1")
    st = _load().orc_solve(n, p, q, _p(X), _p(Y), lamL, lamT, tol, max_iter, stall_iters,
                           int(lambda_passes), int(warm), _p(Lam), _p(Th), ctypes.byref(iters), ctypes.byref(f),
                           ctypes.byref(tr))
    k = iters.value + 1
    trace = {key: v[:k].copy() for key, v in arrs.items()}
    return SolveResult(Lambda=Lam, Theta=Th, f=f.value, iters=iters.value, status=st,
                       trace=trace)
