"""Python access to the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product package never imports this
module and shares no code with it.
"""
from __future__ import annotations

import contextlib
import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

STATUS = {1: "solved", 2: "primal_infeasible", 3: "dual_infeasible",
          4: "max_iter_reached", 5: "time_limit_reached", 6: "unsolved"}


def build(src: str = _SRC, out: str = _SO) -> str:
    """Compile oracle.c (or another copy of it, `src`) into a shared library
    (plain gcc, -O3, no CPU-specific flags)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-D_POSIX_C_SOURCE=200809L",
                           "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
                           "-I", _HERE, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("m", ctypes.c_int),
                ("P_indptr", ctypes.c_void_p), ("P_indices", ctypes.c_void_p),
                ("P_data", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("A_indptr", ctypes.c_void_p), ("A_indices", ctypes.c_void_p),
                ("A_data", ctypes.c_void_p), ("l", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class _Settings(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("rho", "sigma", "alpha", "eps_abs", "eps_rel", "eps_pinf", "eps_dinf",
                 "delta", "time_limit")] + \
               [(k, ctypes.c_int) for k in
                ("max_iter", "check_every", "scaling_iters", "adaptive_rho", "polish",
                 "polish_refine_iter")]


class _Info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("status", "iter", "rho_updates", "polish_status")] + \
               [(k, ctypes.c_double) for k in
                ("obj_val", "prim_res", "dual_res", "eps_prim", "eps_dual", "rho_bar",
                 "setup_time", "solve_time", "polish_time")]


_lib = None


def _open(path: str):
    lib = ctypes.CDLL(path)
    lib.orc_solve.restype = ctypes.c_int
    lib.orc_ldl_solve.restype = ctypes.c_int
    lib.orc_mindeg.restype = ctypes.c_int
    lib.orc_ruiz.restype = ctypes.c_int
    lib.orc_rho_update.restype = ctypes.c_double
    lib.orc_rho_update.argtypes = [ctypes.c_double] * 5
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = _open(_SO)
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Run the oracle functions of this module on another build of the
    oracle (a copy with a planted mistake, for the tests that check that the
    pins catch it); the usual library is restored afterwards."""
    global _lib
    saved = _lib
    _lib = _open(path)
    try:
        yield
    finally:
        _lib = saved


def default_settings() -> dict:
    s = _Settings()
    _load().orc_default_settings(ctypes.byref(s))
    return {k: getattr(s, k) for k, _ in _Settings._fields_}


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    status: str
    iter: int
    rho_updates: int
    polish_status: int
    obj_val: float
    prim_res: float
    dual_res: float
    eps_prim: float
    eps_dual: float
    rho_bar: float
    setup_time: float
    solve_time: float
    polish_time: float


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Arrays:
    """Keeps contiguous typed copies alive for the duration of a call."""

    def __init__(self, qp):
        P = qp.P.tocsr()
        A = qp.A.tocsr()
        self.n, self.m = P.shape[0], A.shape[0]
        self.Pp = np.ascontiguousarray(P.indptr, dtype=np.int32)
        self.Pi = np.ascontiguousarray(P.indices, dtype=np.int32)
        self.Px = np.ascontiguousarray(P.data, dtype=np.float64)
        self.Ap = np.ascontiguousarray(A.indptr, dtype=np.int32)
        self.Ai = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.Ax = np.ascontiguousarray(A.data, dtype=np.float64)
        self.q = np.ascontiguousarray(qp.q, dtype=np.float64)
        self.l = np.ascontiguousarray(qp.l, dtype=np.float64)
        self.u = np.ascontiguousarray(qp.u, dtype=np.float64)

    def problem(self):
        return _Problem(self.n, self.m, _ptr(self.Pp), _ptr(self.Pi), _ptr(self.Px),
                        _ptr(self.q), _ptr(self.Ap), _ptr(self.Ai), _ptr(self.Ax),
                        _ptr(self.l), _ptr(self.u))


def solve(qp, x_ws=None, y_ws=None, **settings) -> Result:
    """Run the oracle on a qpgen.QP; keyword arguments override settings."""
    lib = _load()
    arr = _Arrays(qp)
    s = _Settings()
    lib.orc_default_settings(ctypes.byref(s))
    for k, v in settings.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    x = np.zeros(arr.n)
    y = np.zeros(max(arr.m, 1))
    z = np.zeros(max(arr.m, 1))
    info = _Info()
    xw = None if x_ws is None else np.ascontiguousarray(x_ws, dtype=np.float64)
    yw = None if y_ws is None else np.ascontiguousarray(y_ws, dtype=np.float64)
    pb = arr.problem()
    rc = lib.orc_solve(ctypes.byref(pb), ctypes.byref(s),
                       _ptr(xw) if xw is not None else None,
                       _ptr(yw) if yw is not None else None,
                       _ptr(x), _ptr(y), _ptr(z), ctypes.byref(info))
    if rc != 0:
        raise RuntimeError(f"oracle failed with code {rc}")
    return Result(x=x, y=y[:arr.m], z=z[:arr.m], status=STATUS[info.status], iter=info.iter,
                  rho_updates=info.rho_updates, polish_status=info.polish_status,
                  obj_val=info.obj_val, prim_res=info.prim_res, dual_res=info.dual_res,
                  eps_prim=info.eps_prim, eps_dual=info.eps_dual, rho_bar=info.rho_bar,
                  setup_time=info.setup_time, solve_time=info.solve_time,
                  polish_time=info.polish_time)


def rho_update(rho_bar: float, prim_res: float, prim_norm: float, dual_res: float,
               dual_norm: float) -> float:
    """The Section 5.2 rho-bar rule the solver applies at each check."""
    return float(_load().orc_rho_update(rho_bar, prim_res, prim_norm, dual_res, dual_norm))


def ruiz(qp, iters: int = 10):
    lib = _load()
    arr = _Arrays(qp)
    D = np.zeros(arr.n)
    E = np.zeros(max(arr.m, 1))
    c = ctypes.c_double(0.0)
    pb = arr.problem()
    lib.orc_ruiz(ctypes.byref(pb), int(iters), _ptr(D), _ptr(E), ctypes.byref(c))
    return D, E[:arr.m], c.value


def ldl_solve(K_upper_csc, b):
    """Solve K x = b, K symmetric quasi-definite given as scipy upper-triangular CSC."""
    lib = _load()
    K = K_upper_csc.tocsc()
    K.sort_indices()
    N = K.shape[0]
    Kp = np.ascontiguousarray(K.indptr, dtype=np.int32)
    Ki = np.ascontiguousarray(K.indices, dtype=np.int32)
    Kx = np.ascontiguousarray(K.data, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(N)
    rc = lib.orc_ldl_solve(N, _ptr(Kp), _ptr(Ki), _ptr(Kx), _ptr(b), _ptr(x))
    if rc != 0:
        raise RuntimeError(f"LDL failed with code {rc}")
    return x


def mindeg(K_upper_csc):
    lib = _load()
    K = K_upper_csc.tocsc()
    N = K.shape[0]
    Kp = np.ascontiguousarray(K.indptr, dtype=np.int32)
    Ki = np.ascontiguousarray(K.indices, dtype=np.int32)
    perm = np.zeros(N, dtype=np.int32)
    rc = lib.orc_mindeg(N, _ptr(Kp), _ptr(Ki), _ptr(perm))
    if rc != 0:
        raise RuntimeError("ordering failed")
    return perm
