"""Degenerate and edge inputs on the GPU through the C ABI, against closed
forms and the oracle: a scalar QP, no constraints at all (m = 0), A = I
(no multi-entry rows, so the dense factor has no rank-k part), a linear
program (P = 0), rows of A that are empty or free (infinite bounds on
both sides), which must not change the solution, and the band factor on
edge patterns (zero bandwidth, a ragged last block, a chain)."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import qpgen
from qpgen import QP
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp64", "fp32"]
# tolerances of the tight solves: the FP32 path is held to the paper's
# high-accuracy setting, the FP64 path one decade further
EPS = {"fp64": 1e-6, "fp32": 1e-5}


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    assert pm.device_count() > 0, "no HIP device"
    return pm


def _qp(P, q, A, l, u, name):
    P = sp.csr_matrix(np.triu(np.atleast_2d(np.asarray(P, float))))
    A = sp.csr_matrix(np.asarray(A, float).reshape(len(l), -1))
    return QP(P, np.asarray(q, float), A, np.asarray(l, float), np.asarray(u, float), name=name)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_scalar_qp(pm, precision):
    """n = m = 1: min x^2 - 4x on [-1, 1] -> x = 1, y = 2 (bound active)."""
    qp = _qp([[2.0]], [-4.0], [[1.0]], [-1.0], [1.0], "scalar")
    print(f"scalar {precision}", flush=True)
    e = EPS[precision]
    x, y, info = pm.solve(qp, precision=precision, eps_abs=e, eps_rel=e)
    gc.compare(qp, x, y, info, oracle.solve(qp, eps_abs=e, eps_rel=e), eps_abs=e, eps_rel=e)
    assert abs(x[0] - 1.0) <= 1e-4 and abs(y[0] - 2.0) <= 1e-3
    assert abs(info["obj_val"] + 3.0) <= 1e-4


@pytest.mark.parametrize("precision", PRECISIONS)
def test_no_constraints(pm, precision):
    """m = 0: x = -P^-1 q, an empty dual."""
    rng = np.random.default_rng(11)
    n = 12
    M = rng.standard_normal((n, n))
    P = M @ M.T + np.eye(n)
    q = rng.standard_normal(n)
    qp = QP(sp.csr_matrix(np.triu(P)), q, sp.csr_matrix((0, n)), np.zeros(0), np.zeros(0),
            name="m=0")
    print(f"m=0 {precision}", flush=True)
    e = EPS[precision]
    x, y, info = pm.solve(qp, precision=precision, eps_abs=e, eps_rel=e)
    assert info["status_name"] == "solved" and y.size == 0
    xs = -np.linalg.solve(P, q)
    assert np.allclose(x, xs, atol=1e-4 * max(1.0, np.abs(xs).max()))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_identity_constraints(pm, precision):
    """A = I, P diagonal: x = clip(-q/d, l, u); no row of A has two entries."""
    rng = np.random.default_rng(12)
    n = 40
    d = rng.uniform(0.1, 10.0, n)
    q = 3 * rng.standard_normal(n)
    l, u = -rng.random(n), rng.random(n)
    qp = qpgen.box_qp(d, q, l, u)
    print(f"A=I {precision}", flush=True)
    e = EPS[precision]
    x, y, info = pm.solve(qp, precision=precision, eps_abs=e, eps_rel=e)
    gc.compare(qp, x, y, info, oracle.solve(qp, eps_abs=e, eps_rel=e), eps_abs=e, eps_rel=e)
    assert np.allclose(x, np.clip(-q / d, l, u), atol=1e-4)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_linear_program(pm, precision):
    """P = 0, A = I, finite box: x_i = l_i where q_i > 0, else u_i."""
    rng = np.random.default_rng(13)
    n = 20
    q = rng.standard_normal(n)
    l, u = -rng.random(n) - 0.1, rng.random(n) + 0.1
    qp = QP(sp.csr_matrix((n, n)), q, sp.identity(n, format="csr"), l, u, name="box LP")
    print(f"LP {precision}", flush=True)
    e = EPS[precision]
    kw = dict(eps_abs=e, eps_rel=e, max_iter=50000)
    x, y, info = pm.solve(qp, precision=precision, **kw)
    gc.compare(qp, x, y, info, oracle.solve(qp, **kw), eps_abs=e, eps_rel=e)
    xs = np.where(q > 0, l, u)
    assert np.allclose(x, xs, atol=1e-3)
    assert abs(info["obj_val"] - q @ xs) <= 1e-3 * max(1.0, abs(q @ xs))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_empty_and_free_rows_change_nothing(pm, precision):
    """Rows without entries (l <= 0 <= u) and rows with infinite bounds on
    both sides added to a random QP: same status, and the objective of the
    base problem's solution."""
    base = qpgen.config_instance(1, 5)
    rng = np.random.default_rng(14)
    k_free = 3
    F = sp.csr_matrix(rng.standard_normal((k_free, base.n)))
    E = sp.csr_matrix((2, base.n))
    A = sp.vstack([base.A, E, F], format="csr")
    l = np.concatenate([base.l, [-1.0, 0.0], -np.inf * np.ones(k_free)])
    u = np.concatenate([base.u, [1.0, 0.0], np.inf * np.ones(k_free)])
    qp = QP(base.P, base.q, A, l, u, name="random + empty + free rows")
    print(f"empty/free rows {precision}", flush=True)
    e = EPS[precision]
    kw = dict(eps_abs=e, eps_rel=e, max_iter=50000)
    xb, yb, ib = pm.solve(base, precision=precision, **kw)
    x, y, info = pm.solve(qp, precision=precision, **kw)
    gc.compare(qp, x, y, info, oracle.solve(qp, **kw), eps_abs=e, eps_rel=e)
    assert info["status_name"] == ib["status_name"] == "solved"
    assert abs(info["obj_val"] - ib["obj_val"]) <= 1e-4 * max(1.0, abs(ib["obj_val"]))
    assert np.allclose(y[base.m:], 0.0, atol=1e-6)


def test_batch_of_degenerate_and_regular_qps(pm):
    """Scalar, m = 0, A = I and LP instances in one batch with regular QPs:
    each result is bitwise the one of its solve alone (one QP per
    workgroup, fixed reduction order)."""
    rng = np.random.default_rng(15)
    n = 6
    M = rng.standard_normal((n, n))
    odd = [
        _qp([[2.0]], [-4.0], [[1.0]], [-1.0], [1.0], "scalar"),
        QP(sp.csr_matrix(np.triu(M @ M.T + np.eye(n))), rng.standard_normal(n),
           sp.csr_matrix((0, n)), np.zeros(0), np.zeros(0), name="m=0"),
        qpgen.box_qp(rng.uniform(0.1, 2.0, 9), rng.standard_normal(9), -np.ones(9), np.ones(9)),
    ]
    regular = [qpgen.config_instance(1, i) for i in range(4)]
    qps = regular[:2] + odd + regular[2:]
    print("degenerate batch", flush=True)
    b = pm.Batch(qps, precision="fp32")
    b.solve()
    mixed = [b.get(i) for i in range(len(qps))]
    b.close()
    for qp, (x, y, info) in zip(qps, mixed):
        xa, ya, ia = pm.solve(qp, precision="fp32")
        assert info["status_name"] == ia["status_name"] == "solved", qp.name
        assert np.array_equal(x, xa) and np.array_equal(y, ya), qp.name


@pytest.mark.parametrize("precision", PRECISIONS)
def test_band_factor_degenerate_bands(pm, precision):
    """The band factor on edge patterns: a diagonal P with no constraints
    (half-bandwidth 0, blocks of 8, a ragged last block) against the closed
    form x = -q / d; and a chain (tridiagonal P, rows x_i - x_{i+1} with
    bounds) with an empty row and a free row added, against the oracle and
    against the chain without those rows."""
    rng = np.random.default_rng(21)
    e = EPS[precision]
    kw = dict(eps_abs=e, eps_rel=e, max_iter=50000)
    n = 43
    d = rng.uniform(0.5, 3.0, n)
    q = rng.standard_normal(n)
    qp = QP(sp.csr_matrix(np.diag(d)), q, sp.csr_matrix((0, n)), np.zeros(0), np.zeros(0),
            name="diag m=0")
    x, y, info = pm.solve(qp, precision=precision, linsys="band", **kw)
    assert info["linsys"] == 4 and info["status_name"] == "solved"
    assert np.allclose(x, -q / d, atol=1e-6)
    # chain
    n = 150
    main = rng.uniform(1.0, 2.0, n)
    off = rng.uniform(-0.4, 0.4, n - 1)
    P = sp.diags([main, off, off], [0, 1, -1]).toarray()
    D = sp.diags([np.ones(n - 1), -np.ones(n - 1)], [0, 1], shape=(n - 1, n)).toarray()
    A = np.vstack([D, np.zeros((1, n)), np.eye(n)[:1]])
    l = np.concatenate([-0.3 * np.ones(n - 1), [-1.0], [-np.inf]])
    u = np.concatenate([0.3 * np.ones(n - 1), [1.0], [np.inf]])
    q = 3.0 * rng.standard_normal(n)
    base = _qp(P, q, D, -0.3 * np.ones(n - 1), 0.3 * np.ones(n - 1), "chain")
    ext = _qp(P, q, A, l, u, "chain + empty + free rows")
    xb, yb, ib = pm.solve(base, precision=precision, **kw)
    x, y, info = pm.solve(ext, precision=precision, **kw)
    assert ib["linsys"] == info["linsys"] == 4
    gc.compare(ext, x, y, info, oracle.solve(ext, **kw), eps_abs=e, eps_rel=e)
    assert info["status_name"] == ib["status_name"] == "solved"
    assert abs(info["obj_val"] - ib["obj_val"]) <= 1e-4 * max(1.0, abs(ib["obj_val"]))
    assert np.allclose(y[n - 1:], 0.0, atol=1e-6)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_failed_factor_falls_back_to_jacobi(pm, precision):
    """A reduced matrix whose FP32 Cholesky meets a zero pivot: P couples two
    variables with weight 1e8 and the box rows add rho = 0.1 to its diagonal,
    which FP32 rounds away (no Ruiz scaling to even it out), so the second
    pivot is 1e8 - 1e8 = 0.  In FP32 the dense path then solves with Jacobi
    PCG, step for step as the Jacobi path does; in FP64 the factor holds and
    each ADMM step is the exact direct step (the oracle's iteration count).
    Both hold the oracle's status and objective."""
    a = 1e8
    P = sp.csr_matrix(np.array([[a, a, 0.0], [0.0, a, 0.0], [0.0, 0.0, 1.0]]))
    qp = QP(P, np.array([1.0, -1.0, 0.5]), sp.csr_matrix(np.eye(3)), -np.ones(3), np.ones(3),
            name="coupled 1e8")
    kw = dict(scaling_iters=0)
    ref = oracle.solve(qp, **kw)
    xd, yd, idn = pm.solve(qp, precision=precision, linsys="dense", **kw)
    xj, yj, ij = pm.solve(qp, precision=precision, linsys="pcg", **kw)
    assert idn["linsys"] == 2 and ij["linsys"] == 1
    for x, y, info in ((xd, yd, idn), (xj, yj, ij)):
        row = gc.compare(qp, x, y, info, ref)
        gc.assert_obj_parity([row], f"{qp.name} {precision} linsys {info['linsys']}")
    if precision == "fp32":
        assert np.array_equal(xd, xj) and np.array_equal(yd, yj)
        assert (idn["iter"], idn["pcg_iter"]) == (ij["iter"], ij["pcg_iter"])
    else:
        assert idn["pcg_iter"] == idn["iter"] == ref.iter


@pytest.mark.parametrize("precision", PRECISIONS)
def test_band_factor_at_its_largest(pm, precision):
    """The band path at its limits: n = 8192 variables (the permuted vector
    of the direct step fills the LDS stage exactly) and half-bandwidth 64
    (the largest block), 128 blocks.  The automatic choice takes the band
    factor; status and objective are the oracle's, and each ADMM step is one
    direct step (in FP64 with the oracle's iteration count)."""
    qp = qpgen.banded(np.random.default_rng(5), 8192, 64)
    ref = oracle.solve(qp)
    x, y, info = pm.solve(qp, precision=precision)
    assert info["linsys"] == 4, info["linsys"]
    row = gc.compare(qp, x, y, info, ref)
    gc.assert_obj_parity([row], f"{qp.name} {precision}")
    assert info["pcg_iter"] == info["iter"]
    if precision == "fp64":
        assert info["iter"] == ref.iter


@pytest.mark.parametrize("linsys", ["pcg", "dense"])
def test_fp32_overflow_is_reported_unsolved(pm, linsys):
    """Finite data whose FP32 products overflow: with q = 1e20 and the
    scaling off, the curvature p'Kp of the first inner step is about 1e40,
    past FP32's range.  The FP32 path then stops at the first check with
    "unsolved" (reading 31) instead of reading infinite or NaN residuals as
    converged.  With Ruiz and cost scaling on, the same QP is solved with the
    oracle's status and objective."""
    qp = QP(sp.csr_matrix(np.eye(3)), 1e20 * np.array([1.0, -1.0, 0.5]),
            sp.csr_matrix(np.eye(3)), -np.ones(3), np.ones(3), name="q = 1e20")
    x, y, info = pm.solve(qp, precision="fp32", linsys=linsys, scaling_iters=0)
    assert info["status_name"] == "unsolved", info["status_name"]
    assert info["iter"] == 25
    x, y, info = pm.solve(qp, precision="fp32", linsys=linsys)
    row = gc.compare(qp, x, y, info, oracle.solve(qp))
    gc.assert_obj_parity([row], f"{qp.name} scaled, linsys {linsys}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_polish_with_a_zero_equality_dual(pm, precision):
    """A degenerate dual: the equality row x_0 = 0 has multiplier 0 at the
    optimum (the unconstrained minimiser already meets it), so its ADMM and
    polished duals are rounding-sized with either sign.  An equality row
    puts no sign condition on its dual (both bounds are active), so the
    device's FP64 polish is accepted as the oracle's is, at the optimum
    known by construction."""
    from tests.test_oracle_pins import _equality_with_zero_dual
    cases = [_equality_with_zero_dual(seed) for seed in range(24)]
    b = pm.Batch([qp for qp, _ in cases], precision=precision, polish=1)
    b.solve()
    for i, (qp, xs) in enumerate(cases):
        x, y, info = b.get(i)
        assert info["status_name"] == "solved" and info["polish_status"] == 1, qp.name
        assert np.max(np.abs(x - xs)) <= 1e-9 * max(1.0, np.max(np.abs(xs))), qp.name
    b.close()
