"""Parametric re-solves on the GPU through the C ABI (Section 6): new matrix
values with the patterns kept, and the paper's parametric workloads in
synthetic form -- a Lasso regularisation path, an MPC closed loop and a
portfolio back test -- each re-solve checked against the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import qpgen
from qpgen import QP
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    assert pm.device_count() > 0, "no HIP device"
    return pm


def _new_values(qp: QP, rng: np.random.Generator, name: str) -> QP:
    """Same patterns: A's entries scaled by U[0.5, 1.5]; P scaled by a
    positive diagonal congruence D P D (stays positive semidefinite)."""
    A = qp.A.copy()
    A.data = A.data * rng.uniform(0.5, 1.5, A.nnz)
    d = rng.uniform(0.7, 1.3, qp.n)
    P = qp.P.tocsr().copy()
    rows = np.repeat(np.arange(qp.n), np.diff(P.indptr))
    P.data = P.data * d[rows] * d[P.indices]
    return QP(P, qp.q.copy(), A, qp.l.copy(), qp.u.copy(), name=name)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_update_matrices_matches_oracle(pm, precision):
    """osqp_batch_update_matrices on a random QP (dense path), an MPC QP and a
    factor-model portfolio (low-rank path) of one batch.  The re-solve starts
    from the last solution with the last rho-bar; the oracle, warm-started
    from the same x, y with the same rho-bar, reaches the same status and
    objective on the modified problems.  A fresh setup of them reaches the
    same statuses."""
    rng = qpgen.rng_for(9, 1)
    qps = [qpgen.config_instance(1, 3), qpgen.config_instance(3, 2),
           qpgen.config_instance(4, 5, n_range=(100, 400))]
    new = [_new_values(q, rng, q.name + "'") for q in qps]
    print(f"update_matrices {precision}", flush=True)
    b = pm.Batch(qps, precision=precision)
    b.solve()
    prev = [b.get(i) for i in range(3)]
    paths = [p[2]["linsys"] for p in prev]
    for i, q in enumerate(new):
        b.update_matrices(i, P=q.P, A=q.A)
    b.solve()
    res = [b.get(i) for i in range(3)]
    b.close()
    assert [r[2]["linsys"] for r in res] == paths
    refs = [oracle.solve(q, x_ws=p[0], y_ws=p[1], rho=p[2]["rho_bar"]) for q, p in zip(new, prev)]
    rows = [gc.compare(q, *r, ref) for q, r, ref in zip(new, res, refs)]
    gc.summarize(rows, f"update_matrices {precision}")
    gc.assert_obj_parity(rows, f"update_matrices {precision}")
    fresh = pm.Batch(new, precision=precision)
    fresh.solve()
    for i, q in enumerate(new):
        assert fresh.get(i)[2]["status"] == res[i][2]["status"]
    fresh.close()


def test_update_matrices_only_one_matrix_and_errors(pm):
    """P alone, then A alone; a different pattern or count is refused."""
    qp = qpgen.config_instance(1, 4)
    q2 = _new_values(qp, qpgen.rng_for(9, 2), "p-only")
    q2 = QP(q2.P, qp.q, qp.A, qp.l, qp.u, name="P only")
    s = pm.Solver(qp, precision="fp32")
    s.solve()
    s.update_matrices(P=q2.P)
    s.solve()
    gc.compare(q2, *s.result(), oracle.solve(q2))
    q3 = _new_values(qp, qpgen.rng_for(9, 3), "a-only")
    q3 = QP(q2.P, qp.q, q3.A, qp.l, qp.u, name="A only")
    s.update_matrices(A=q3.A)
    s.solve()
    gc.compare(q3, *s.result(), oracle.solve(q3))
    bad = qp.A.tolil()
    bad[0, 0] = 0.0 if qp.A[0, 0] != 0.0 else 1.0
    with pytest.raises(ValueError):
        s.update_matrices(A=sp.csr_matrix(bad))
    import ctypes
    L = pm.lib()
    a = np.ones(3)
    assert L.osqp_batch_update_matrices(s._h, 0, None, 0, ctypes.c_void_p(a.ctypes.data), 3) == 1
    s.close()


def test_lasso_regularisation_path(pm):
    """Lasso path: lambda decreasing over six values, q updated and the
    previous iterate kept (warm start); every point matches the oracle, and
    the warm-started path needs fewer iterations than cold solves."""
    base = qpgen.lasso(qpgen.rng_for(2, 7), 40, 400, density=0.15, lam_frac=1.0)
    lam_max = base.lam
    fr = [0.8, 0.6, 0.45, 0.3, 0.2, 0.1]
    warm = pm.Solver(base, precision="fp32")
    warm.solve()
    it_warm = it_cold = 0
    nf = 40
    for f in fr:
        q = base.q.copy()
        q[-nf:] = f * lam_max
        qp = QP(base.P, q, base.A, base.l, base.u, name=f"lasso lam={f:g} lam_max")
        warm.update_vectors(q=q)
        warm.solve()
        x, y, info = warm.result()
        gc.compare(qp, x, y, info, oracle.solve(qp))
        it_warm += info["iter"]
        _, _, ci = pm.solve(qp, precision="fp32")
        it_cold += ci["iter"]
    warm.close()
    print(f"lasso path: warm {it_warm} iterations, cold {it_cold}", flush=True)
    assert it_warm < it_cold


def test_mpc_closed_loop(pm):
    """MPC closed loop: at each of eight steps the first input is applied to
    the plant, the initial-state rows get the new state (update_vectors of
    l, u) and the re-solve is warm; every step matches the oracle."""
    rng = qpgen.rng_for(3, 900)
    plant = qpgen.mpc_plant(rng)
    Ad, B = plant[0], plant[1]
    nx, nu, T = 20, 10, 10
    x = rng.uniform(-1.0, 1.0, nx)
    qp = qpgen.mpc(rng, T=T, plant=plant, x_init=x)
    s = pm.Solver(qp, precision="fp32")
    its = []
    for step in range(8):
        s.solve()
        xs, ys, info = s.result()
        gc.compare(qp, xs, ys, info, oracle.solve(qp))
        its.append(info["iter"])
        u0 = xs[nx * (T + 1): nx * (T + 1) + nu]
        x = Ad @ x + B @ u0
        qp = qpgen.mpc(rng, T=T, plant=plant, x_init=x)
        s.update_vectors(l=qp.l, u=qp.u)
    s.close()
    print(f"mpc closed loop iterations {its}", flush=True)


def test_portfolio_back_test(pm):
    """Portfolio back test: the factor model stays, the expected returns move
    each period (q updated, warm start); every period matches the oracle."""
    rng = qpgen.rng_for(4, 900)
    F, Dd, mu = qpgen.portfolio_model(rng, 300)
    s = None
    its = []
    for period in range(6):
        mu = 0.8 * mu + 0.2 * rng.standard_normal(mu.size)
        qp = qpgen.portfolio(rng, model=(F, Dd, mu))
        if s is None:
            s = pm.Solver(qp, precision="fp32")
        else:
            s.update_vectors(q=qp.q)
        s.solve()
        xs, ys, info = s.result()
        gc.compare(qp, xs, ys, info, oracle.solve(qp))
        its.append(info["iter"])
    s.close()
    print(f"portfolio back test iterations {its}", flush=True)
