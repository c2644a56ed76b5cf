"""Python binding of osqp_mi, the MI355X (gfx950) implementation of the
operator-splitting ADMM QP method (OSQP paper).

This module only marshals arguments into the C ABI of libosqp_mi.so
(include/osqp_mi.h); every step of the solve runs in the library's HIP
kernels.  There is no CPU fallback: a missing library or device raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libosqp_mi.so")

STATUS = {1: "solved", 2: "primal_infeasible", 3: "dual_infeasible",
          4: "max_iter_reached", 5: "time_limit_reached", 6: "unsolved"}
ERRORS = {0: "ok", 1: "dim", 2: "csr", 3: "p_not_upper", 4: "data_nonfinite", 5: "l_gt_u",
          6: "settings", 7: "alloc", 8: "budget", 9: "device", 10: "not_setup",
          11: "index", 12: "no_device", 13: "unsupported"}
PRECISION = {"fp64": 0, "fp32": 1}
LINSYS = {"auto": 0, "pcg": 1, "dense": 2, "lowrank": 3, "band": 4}

# every function the header declares (the CPU tests check the exports)
EXPORTS = [
    "osqp_set_default_settings", "osqp_error_string", "osqp_set_allocator", "osqp_device_count",
    "osqp_device_info", "osqp_setup",
    "osqp_solve", "osqp_update_vectors", "osqp_warm_start", "osqp_update_matrices",
    "osqp_get_solution",
    "osqp_get_info", "osqp_cleanup", "osqp_batch_setup", "osqp_batch_solve",
    "osqp_batch_solve_async", "osqp_batch_solve_subset_async", "osqp_batch_sync",
    "osqp_batch_solve_graph_async", "osqp_batch_autotune", "osqp_batch_set_shape",
    "osqp_batch_reset",
    "osqp_batch_update_vectors", "osqp_batch_warm_start", "osqp_batch_update_matrices",
    "osqp_batch_get",
    "osqp_batch_last_kernel_ms", "osqp_batch_count", "osqp_batch_get_factor",
    "osqp_batch_cleanup", "osqp_server_create", "osqp_server_submit", "osqp_server_wait",
    "osqp_server_stats", "osqp_server_destroy",
]


class OSQPError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: error {code} ({ERRORS.get(code, '?')})")


class _Csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int32), ("ncols", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("data", ctypes.c_void_p)]


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("P_upper", _Csr),
                ("q", ctypes.c_void_p), ("A", _Csr), ("l", ctypes.c_void_p),
                ("u", ctypes.c_void_p)]


_SET_F = ["rho", "sigma", "alpha", "eps_abs", "eps_rel", "eps_prim_inf", "eps_dual_inf",
          "delta", "time_limit", "pcg_tol_frac"]
_SET_I = ["max_iter", "check_every", "scaling_iters", "adaptive_rho", "polish",
          "polish_refine_iter", "precision", "linsys", "pcg_max_iter", "block_size"]


class _Settings(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in _SET_F] + \
               [(k, ctypes.c_int32) for k in _SET_I] + [("stream", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in
                ("status", "iter", "pcg_iter", "rho_updates", "polish_status", "linsys")] + \
               [(k, ctypes.c_double) for k in
                ("obj_val", "prim_res", "dual_res", "eps_prim", "eps_dual", "rho_bar",
                 "setup_time", "solve_time", "polish_time", "factor_time", "pcg_time",
                 "update_time", "check_time")]


class _Tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("block_size", "lane_div", "trials")] + \
               [(k, ctypes.c_double) for k in ("default_ms", "best_ms")]


# device-memory callbacks of osqp_set_allocator: alloc(bytes, ctx) -> pointer,
# free(pointer, ctx)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None   # the installed callbacks
_allocator_history = []  # every pair installed, kept callable for the process

_lib = None


def lib() -> ctypes.CDLL:
    """Load libosqp_mi.so (built by paper_1711_08013_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1711_08013_amd/build.py")
        _lib = _configure(ctypes.CDLL(LIB_PATH))
    return _lib


def _configure(L: ctypes.CDLL) -> ctypes.CDLL:
    """Checks that every exported function is there and sets the result and
    argument types the C ABI declares."""
    for name in EXPORTS:
        getattr(L, name)
    L.osqp_error_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("osqp_error_string", "osqp_cleanup", "osqp_batch_cleanup",
                        "osqp_server_destroy"):
            getattr(L, name).restype = ctypes.c_int32
    L.osqp_cleanup.restype = None
    L.osqp_batch_cleanup.restype = None
    L.osqp_server_destroy.restype = None
    L.osqp_server_create.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                     ctypes.c_void_p]
    L.osqp_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.osqp_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.osqp_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, ctypes.c_void_p]
    return L


def set_allocator(alloc=None, free=None):
    """Device memory of the handles created from now on comes from
    alloc(nbytes) -> int address and goes back through free(address)
    (osqp_set_allocator); no arguments restore hipMalloc / hipFree."""
    global _allocator_refs
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check(lib().osqp_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "osqp_set_allocator")
        _allocator_refs = None
        return

    def _a(nbytes, _ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:   # an exception must not cross the C boundary
            return None

    def _f(ptr, _ctx):
        try:
            free(int(ptr))
        except Exception:
            pass

    refs = (_ALLOC_FN(_a), _FREE_FN(_f))
    _check(lib().osqp_set_allocator(refs[0], refs[1], None), "osqp_set_allocator")
    _allocator_refs = refs
    # a handle frees through the pair it was created with, also after another
    # pair (or none) is installed: every pair stays callable for the process
    _allocator_history.append(refs)


def use_torch_allocator(device: int = 0):
    """Device memory from PyTorch's caching allocator (on `device`, torch's
    current stream), so the solver's memory is counted and reused with the
    caller's tensors; torch.cuda.current_stream().cuda_stream can be passed as
    the `stream` setting to run on torch's stream as well."""
    import torch
    set_allocator(lambda nb: torch.cuda.caching_allocator_alloc(nb, device),
                  torch.cuda.caching_allocator_delete)


def device_count() -> int:
    return int(lib().osqp_device_count())


def device_info() -> dict:
    v = [ctypes.c_int32(0) for _ in range(4)]
    _check(lib().osqp_device_info(*[ctypes.byref(x) for x in v]), "osqp_device_info")
    return dict(zip(("cu_count", "lds_per_block", "lds_per_cu", "wall_khz"), (x.value for x in v)))


def default_settings() -> dict:
    s = _Settings()
    lib().osqp_set_default_settings(ctypes.byref(s))
    return {k: getattr(s, k) for k in _SET_F + _SET_I}


def _make_settings(kw: dict) -> _Settings:
    s = _Settings()
    lib().osqp_set_default_settings(ctypes.byref(s))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "linsys" and isinstance(v, str):
            v = LINSYS[v]
        if k == "stream":
            s.stream = None if v is None else ctypes.c_void_p(int(v))
            continue
        if k not in _SET_F and k not in _SET_I:
            raise KeyError(f"unknown setting {k}")
        setattr(s, k, v)
    return s


def _ptr(a) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _canonical_csr(M):
    """CSR copy with duplicates summed and each row's columns sorted (the C ABI
    requires strictly increasing columns); explicit zeros are kept, since
    they belong to the pattern that later value updates refer to."""
    import scipy.sparse as sp
    C = sp.csr_matrix(M, copy=True)
    C.sum_duplicates()
    C.sort_indices()
    return C


class _Keep:
    """Typed contiguous copies of one QP's arrays, kept alive during a call."""

    def __init__(self, qp):
        P = _canonical_csr(qp.P)
        A = _canonical_csr(qp.A)
        self.n, self.m = int(P.shape[0]), int(A.shape[0])
        self.Pp = np.ascontiguousarray(P.indptr, dtype=np.int32)
        self.Pi = np.ascontiguousarray(P.indices, dtype=np.int32)
        self.Px = np.ascontiguousarray(P.data, dtype=np.float64)
        self.Ap = np.ascontiguousarray(A.indptr, dtype=np.int32)
        self.Ai = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.Ax = np.ascontiguousarray(A.data, dtype=np.float64)
        self.q = np.ascontiguousarray(qp.q, dtype=np.float64)
        self.l = np.ascontiguousarray(qp.l, dtype=np.float64)
        self.u = np.ascontiguousarray(qp.u, dtype=np.float64)
        self.pnnz, self.annz = int(P.nnz), int(A.nnz)

    def problem(self) -> _Problem:
        Pc = _Csr(self.n, self.n, self.pnnz, _ptr(self.Pp), _ptr(self.Pi), _ptr(self.Px))
        Ac = _Csr(self.m, self.n, self.annz, _ptr(self.Ap), _ptr(self.Ai), _ptr(self.Ax))
        return _Problem(self.n, self.m, Pc, _ptr(self.q), Ac, _ptr(self.l), _ptr(self.u))


def _check(rc: int, where: str):
    if rc != 0:
        raise OSQPError(int(rc), where)


def _info_dict(info: _Info) -> dict:
    d = {k: getattr(info, k) for k, _ in _Info._fields_}
    d["status_name"] = STATUS.get(d["status"], "?")
    return d


class Batch:
    """A batch of independent QPs solved together on the GPU (a single QP is a
    batch of one).  `qps` are objects with P (upper-triangular scipy CSR), q,
    A (scipy CSR), l, u."""

    def __init__(self, qps: Sequence, **settings):
        L = lib()
        self._keep = [_Keep(qp) for qp in qps]
        probs = (_Problem * len(self._keep))(*[k.problem() for k in self._keep])
        self._settings = _make_settings(settings)
        h = ctypes.c_void_p()
        _check(L.osqp_batch_setup(ctypes.byref(h), len(self._keep), probs,
                                  ctypes.byref(self._settings)), "osqp_batch_setup")
        self._h = h
        self.sizes = [(k.n, k.m) for k in self._keep]

    def __len__(self):
        return len(self._keep)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def _index(self, i: int) -> int:
        if not 0 <= i < len(self._keep):
            raise IndexError(f"problem index {i} outside 0..{len(self._keep) - 1}")
        return i

    def solve(self):
        _check(lib().osqp_batch_solve(self._h), "osqp_batch_solve")

    def solve_async(self):
        _check(lib().osqp_batch_solve_async(self._h), "osqp_batch_solve_async")

    def solve_subset(self, indices):
        """Solve only the listed QPs (the others keep their state)."""
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        _check(lib().osqp_batch_solve_subset_async(
            self._h, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(idx.size)),
            "osqp_batch_solve_subset_async")
        self.sync()

    def sync(self):
        _check(lib().osqp_batch_sync(self._h), "osqp_batch_sync")

    def solve_graph(self):
        """Solve through the replayable graph of the solve launches."""
        _check(lib().osqp_batch_solve_graph_async(self._h), "osqp_batch_solve_graph_async")
        self.sync()

    def autotune(self, reps: int = 1) -> dict:
        """Time the launch shapes on this batch and keep the fastest (resets it)."""
        t = _Tuning()
        _check(lib().osqp_batch_autotune(self._h, int(reps), ctypes.byref(t)),
               "osqp_batch_autotune")
        return {k: getattr(t, k) for k, _ in _Tuning._fields_}

    def set_shape(self, block_size: int, lane_div: int):
        """Apply a launch shape (workgroup size, lane divisor) directly."""
        _check(lib().osqp_batch_set_shape(self._h, int(block_size), int(lane_div)),
               "osqp_batch_set_shape")

    def reset(self):
        _check(lib().osqp_batch_reset(self._h), "osqp_batch_reset")

    def update_vectors(self, i: int, q=None, l=None, u=None):
        n, m = self.sizes[self._index(i)]
        qa = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        la = None if l is None else np.ascontiguousarray(l, dtype=np.float64)
        ua = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        for a, k in ((qa, n), (la, m), (ua, m)):
            if a is not None and a.size != k:
                raise ValueError("vector size mismatch")
        _check(lib().osqp_batch_update_vectors(self._h, i, _ptr(qa), _ptr(la), _ptr(ua)),
               "osqp_batch_update_vectors")

    def update_matrices(self, i: int, P=None, A=None):
        """New values of P (upper triangle) and/or A with the setup's patterns
        (scipy sparse); the next solve rescales, refactors and warm-starts."""
        k = self._keep[self._index(i)]
        pa = aa = None
        if P is not None:
            P = _canonical_csr(P)
            if not (np.array_equal(P.indptr, k.Pp) and np.array_equal(P.indices, k.Pi)):
                raise ValueError("P pattern differs from the setup's")
            pa = np.ascontiguousarray(P.data, dtype=np.float64)
        if A is not None:
            A = _canonical_csr(A)
            if not (np.array_equal(A.indptr, k.Ap) and np.array_equal(A.indices, k.Ai)):
                raise ValueError("A pattern differs from the setup's")
            aa = np.ascontiguousarray(A.data, dtype=np.float64)
        _check(lib().osqp_batch_update_matrices(self._h, i, _ptr(pa), 0 if pa is None else pa.size,
                                                _ptr(aa), 0 if aa is None else aa.size),
               "osqp_batch_update_matrices")

    def warm_start(self, i: int, x=None, y=None):
        n, m = self.sizes[self._index(i)]
        xa = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        ya = None if y is None else np.ascontiguousarray(y, dtype=np.float64)
        if (xa is not None and xa.size != n) or (ya is not None and ya.size != m):
            raise ValueError("vector size mismatch")
        _check(lib().osqp_batch_warm_start(self._h, i, _ptr(xa), _ptr(ya)),
               "osqp_batch_warm_start")

    def get(self, i: int):
        n, m = self.sizes[self._index(i)]
        x = np.zeros(n)
        y = np.zeros(max(m, 1))
        info = _Info()
        _check(lib().osqp_batch_get(self._h, i, _ptr(x), _ptr(y), ctypes.byref(info)),
               "osqp_batch_get")
        return x, y[:m], _info_dict(info)

    def factor(self, i: int):
        """A factor G (n x n) of problem i's reduced matrix, G G' = K: the
        dense Cholesky factor (lower) or, on the band path, the block-
        bidiagonal factor of the reordered matrix with its rows in variable
        order (osqp_batch_get_factor)."""
        n, _ = self.sizes[self._index(i)]
        L = np.zeros((n, n))
        _check(lib().osqp_batch_get_factor(self._h, i, _ptr(L)), "osqp_batch_get_factor")
        return L

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().osqp_batch_last_kernel_ms(self._h, ctypes.byref(ms)),
               "osqp_batch_last_kernel_ms")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            lib().osqp_batch_cleanup(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server: submit QPs (optionally with a structure key
    shared by QPs with equal P and A), then wait for each ticket."""

    def __init__(self, hbm_budget_bytes: int = 64 << 30, max_slots: int = 1024, **settings):
        self._settings = _make_settings(settings)
        h = ctypes.c_void_p()
        _check(lib().osqp_server_create(ctypes.byref(h), int(hbm_budget_bytes), int(max_slots),
                                        ctypes.byref(self._settings)), "osqp_server_create")
        self._h = h
        self._sizes = {}

    def submit(self, qp, key: int = 0, x_ws=None, y_ws=None) -> int:
        k = _Keep(qp)
        p = k.problem()
        xa = None if x_ws is None else np.ascontiguousarray(x_ws, dtype=np.float64)
        ya = None if y_ws is None else np.ascontiguousarray(y_ws, dtype=np.float64)
        t = ctypes.c_uint64(0)
        _check(lib().osqp_server_submit(self._h, ctypes.byref(p), ctypes.c_uint64(int(key)),
                                        _ptr(xa), _ptr(ya), ctypes.byref(t)), "osqp_server_submit")
        self._sizes[t.value] = (k.n, k.m)
        return t.value

    def wait(self, ticket: int):
        if ticket not in self._sizes:   # never issued here, or already collected
            raise OSQPError(11, "osqp_server_wait")
        n, m = self._sizes[ticket]
        x = np.zeros(n)
        y = np.zeros(max(m, 1))
        info = _Info()
        lat = ctypes.c_double(0.0)
        _check(lib().osqp_server_wait(self._h, ctypes.c_uint64(ticket), _ptr(x), _ptr(y),
                                      ctypes.byref(info), ctypes.byref(lat)), "osqp_server_wait")
        del self._sizes[ticket]
        return x, y[:m], _info_dict(info), lat.value

    def stats(self) -> dict:
        v = [ctypes.c_int64(0) for _ in range(4)]
        _check(lib().osqp_server_stats(self._h, *[ctypes.byref(x) for x in v]),
               "osqp_server_stats")
        return dict(zip(("completed", "batches", "peak_inflight", "peak_bytes"),
                        (x.value for x in v)))

    def close(self):
        if getattr(self, "_h", None):
            lib().osqp_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver(Batch):
    """One QP (osqp_setup / osqp_solve / osqp_update_vectors / osqp_warm_start)."""

    def __init__(self, qp, **settings):
        super().__init__([qp], **settings)

    def update_vectors(self, q=None, l=None, u=None):
        super().update_vectors(0, q, l, u)

    def warm_start(self, x=None, y=None):
        super().warm_start(0, x, y)

    def update_matrices(self, P=None, A=None):
        super().update_matrices(0, P, A)

    def result(self):
        return super().get(0)


def solve(qp, **settings):
    """Convenience: set up, solve and return (x, y, info) for one QP."""
    s = Solver(qp, **settings)
    try:
        s.solve()
        return s.result()
    finally:
        s.close()
