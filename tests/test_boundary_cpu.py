"""CPU-only checks of the C-ABI boundary: the library builds and loads, it
exports every function include/osqp_mi.h declares, defaults follow the
paper, and input validation returns the documented error codes (validation
runs before any device call, so these need no GPU)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen
from qpgen import QP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "osqp_mi.h")


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    if not os.path.exists(pm.LIB_PATH):
        from paper_1711_08013_amd import build
        build.build()
    pm.lib()
    return pm


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:osqp_int|void|const char \*)\s*\*?\s*(osqp_\w+)\s*\(",
                                 txt, re.M)))


def test_header_declares_the_named_entry_points():
    names = _declared()
    for n in ("osqp_setup", "osqp_solve", "osqp_update_vectors", "osqp_warm_start"):
        assert n in names


def test_library_exports_every_declared_symbol(pm):
    lib = pm.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(pm.EXPORTS) == sorted(n for n in _declared() if n in pm.EXPORTS)
    assert set(_declared()) <= set(pm.EXPORTS)


def test_defaults_follow_the_paper(pm):
    s = pm.default_settings()
    assert s["sigma"] == 1e-6 and s["alpha"] == 1.6 and s["rho"] == 0.1
    assert s["eps_abs"] == 1e-3 and s["eps_rel"] == 1e-3
    assert s["eps_prim_inf"] == 1e-4 and s["eps_dual_inf"] == 1e-4
    assert s["polish_refine_iter"] == 3 and s["delta"] == 1e-6
    assert s["check_every"] == 25 and s["scaling_iters"] == 10


def _small():
    return qpgen.random_qp(5, qpgen.rng_for(9, 77))


def _code(pm, fn):
    with pytest.raises(pm.OSQPError) as e:
        fn()
    return e.value.code


def test_validation_codes(pm):
    base = _small()
    # l > u
    qp = _small()
    qp.l = qp.l.copy(); qp.l[0] = qp.u[0] + 1.0
    assert _code(pm, lambda: pm.Batch([qp])) == 5
    # NaN in q
    qp = _small(); qp.q = qp.q.copy(); qp.q[1] = np.nan
    assert _code(pm, lambda: pm.Batch([qp])) == 4
    # NaN in A data
    qp = _small(); A = qp.A.copy(); A.data[0] = np.nan; qp.A = A
    assert _code(pm, lambda: pm.Batch([qp])) == 4
    # NaN bound
    qp = _small(); qp.u = qp.u.copy(); qp.u[2] = np.nan
    assert _code(pm, lambda: pm.Batch([qp])) == 4
    # strictly-lower entry in P
    qp = _small(); qp.P = sp.csr_matrix(qp.full_P())
    assert _code(pm, lambda: pm.Batch([qp])) == 3
    # unsorted / out-of-range CSR
    qp = _small(); A = qp.A.copy()
    A.indices = A.indices.copy(); A.indices[0] = 99
    qp.A = A
    assert _code(pm, lambda: pm.Batch([qp])) == 2
    # settings
    for bad in ({"sigma": 0.0}, {"rho": -1.0}, {"alpha": 2.0}, {"alpha": 0.0},
                {"eps_abs": -1.0}, {"max_iter": 0}, {"check_every": 0},
                {"block_size": 100}, {"precision": 7}):
        assert _code(pm, lambda: pm.Batch([base], **bad)) == 6, bad


def test_empty_batch_and_bad_dims(pm):
    L = pm.lib()
    h = ctypes.c_void_p()
    assert L.osqp_batch_setup(ctypes.byref(h), 0, None, None) == 1
    assert L.osqp_batch_setup(None, 1, None, None) == 10


def test_no_device_is_reported(pm):
    if pm.device_count() > 0:
        pytest.skip("a device is visible")
    with pytest.raises(pm.OSQPError) as e:
        pm.Batch([_small()])
    assert e.value.code == 12


def test_handle_functions_reject_null(pm):
    L = pm.lib()
    assert L.osqp_solve(None) == 10
    assert L.osqp_batch_solve(None) == 10
    assert L.osqp_update_vectors(None, None, None, None) == 10
    assert L.osqp_warm_start(None, None, None) == 10
    assert L.osqp_batch_solve_graph_async(None) == 10
    assert L.osqp_batch_autotune(None, 1, None) == 10
    assert L.osqp_batch_set_shape(None, 256, 16) == 10
    assert L.osqp_update_matrices(None, None, 0, None, 0) == 10
    assert L.osqp_batch_update_matrices(None, 0, None, 0, None, 0) == 10
    L.osqp_cleanup(None)
    L.osqp_batch_cleanup(None)


def test_binding_canonicalises_csr_input(pm):
    """The binding hands the C ABI sorted, duplicate-free rows (which its
    validation requires) without dropping explicit zeros of the pattern."""
    # row 0 given with columns out of order and a duplicate, row 1 with an
    # explicit zero
    indptr = np.array([0, 3, 5])
    indices = np.array([2, 0, 2, 1, 2])
    data = np.array([1.0, 2.0, 3.0, 0.0, 5.0])
    M = sp.csr_matrix((data, indices, indptr), shape=(2, 3))
    C = pm._canonical_csr(M)
    assert C.indptr.tolist() == [0, 2, 4]
    assert C.indices.tolist() == [0, 2, 1, 2]
    assert C.data.tolist() == [2.0, 4.0, 0.0, 5.0]
    # the input is left as it was
    assert M.indices.tolist() == [2, 0, 2, 1, 2]
    P = sp.csr_matrix((np.array([1.0, 0.5, 2.0]), np.array([1, 0, 1]), np.array([0, 2, 3])),
                      shape=(2, 2))
    k = pm._Keep(QP(P, np.zeros(2), sp.csr_matrix(np.eye(2)), -np.ones(2), np.ones(2)))
    assert k.Pi.tolist() == [0, 1, 1] and k.Px.tolist() == [0.5, 1.0, 2.0]


def test_set_allocator_pairs(pm):
    """osqp_set_allocator needs both callbacks or neither (no device call)."""
    L = pm.lib()
    alloc = pm._ALLOC_FN(lambda n, c: None)
    assert L.osqp_set_allocator(alloc, pm._FREE_FN(), None) == 6
    assert L.osqp_set_allocator(pm._ALLOC_FN(), pm._FREE_FN(lambda p, c: None), None) == 6
    assert L.osqp_set_allocator(pm._ALLOC_FN(), pm._FREE_FN(), None) == 0
    with pytest.raises(ValueError):
        pm.set_allocator(lambda n: 0, None)
    pm.set_allocator()
