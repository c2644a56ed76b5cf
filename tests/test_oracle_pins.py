"""Pins of the FP64 CPU oracle to things other than itself: brute-force
active sets, closed forms, the paper's iterative-refinement equivalence,
certificate definitions, hand-solved fixtures and invariants.  CPU only."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen
from qpgen import QP
from tests import qpcheck

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _qp_dense(P, q, A, l, u, name=""):
    P = np.atleast_2d(np.asarray(P, float))
    A = np.atleast_2d(np.asarray(A, float))
    return QP(sp.csr_matrix(np.triu(P)), np.asarray(q, float), sp.csr_matrix(A),
              np.asarray(l, float), np.asarray(u, float), name=name)


# ---------------------------------------------------------------- LDL / ordering
@pytest.mark.parametrize("seed", range(6))
def test_ldl_matches_dense_solve(oracle_lib, seed):
    """Section 3.1: LDL' of the quasi-definite KKT matrix solves eq. kkt;
    checked against a dense LAPACK solve."""
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(3, 60)), int(rng.integers(0, 80))
    M = qpgen.sparse_normal(rng, n, n, 0.2)
    P = (M @ M.T).toarray()
    A = qpgen.sparse_normal(rng, m, n, 0.2).toarray()
    rho = rng.uniform(0.05, 50.0, m)
    Ku, K = qpcheck.kkt_upper(P, A, 1e-6, rho)
    b = rng.standard_normal(n + m)
    x = oracle_lib.ldl_solve(Ku, b)
    xd = np.linalg.solve(K, b)
    assert np.max(np.abs(K @ x - b)) <= 1e-10 * (np.max(np.abs(b)) + 1.0) * max(1.0, np.abs(K).max())
    assert np.allclose(x, xd, rtol=1e-8, atol=1e-8)


def test_mindeg_is_permutation(oracle_lib):
    rng = np.random.default_rng(7)
    A = qpgen.sparse_normal(rng, 300, 120, 0.05).toarray()
    Ku, _ = qpcheck.kkt_upper(np.eye(120), A, 1e-6, np.ones(300))
    perm = oracle_lib.mindeg(Ku)
    assert sorted(perm.tolist()) == list(range(420))


# ---------------------------------------------------------------- hand fixtures
def _read_golden():
    blocks, cur = [], None
    with open(os.path.join(GOLDEN, "tiny_qps.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "name":
                cur = {"name": rest}
                blocks.append(cur)
                continue

            def vec(s):
                return np.array([float(t) for t in s.split()])
            if key in ("P", "A"):
                cur[key] = np.array([vec(r) for r in rest.split(";")])
            elif key == "dims":
                cur["n"], cur["m"] = (int(t) for t in rest.split())
            else:
                cur[key] = vec(rest)
    return blocks


@pytest.mark.parametrize("case", _read_golden(), ids=lambda c: c["name"])
def test_hand_solved(oracle_lib, case):
    qp = _qp_dense(case["P"], case["q"], case["A"], case["l"], case["u"], case["name"])
    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, polish=1, max_iter=20000)
    assert r.status == "solved"
    assert abs(r.obj_val - case["f"][0]) <= 1e-7 * max(1.0, abs(case["f"][0]))
    assert np.allclose(r.x, case["x"], atol=1e-6)
    assert np.allclose(r.y, case["y"], atol=1e-6)
    # the same problem at the default tolerance: objective within 1e-3
    r3 = oracle_lib.solve(qp)
    assert r3.status == "solved"
    assert qpcheck.rel_obj_err(r3.obj_val, case["f"][0]) <= 1e-3


# ---------------------------------------------------------------- brute force
def _tiny_random(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 7))
    m = int(rng.integers(1, 9))
    M = rng.standard_normal((n, n))
    P = M @ M.T + 0.1 * np.eye(n)
    q = rng.standard_normal(n)
    A = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.7)
    l = -rng.random(m)
    u = rng.random(m)
    # some one-sided, free and equality rows
    kind = rng.integers(0, 5, m)
    l[kind == 1] = -np.inf
    u[kind == 2] = np.inf
    eq = kind == 3
    l[eq] = u[eq] = 0.0
    return _qp_dense(P, q, A, l, u, f"tiny{seed}")


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_active_sets(oracle_lib, seed):
    """Section 2 optimality conditions: the optimum from enumerating every
    active set must match the oracle (1e-3 relative at eps = 1e-3; 1e-7 with
    tight tolerances and polishing)."""
    qp = _tiny_random(seed)
    bf = qpcheck.brute_force(qp)
    assert bf is not None  # x = 0 is feasible, P > 0: a solution exists
    x_bf, y_bf, f_bf = bf
    r = oracle_lib.solve(qp)
    assert r.status == "solved"
    assert qpcheck.rel_obj_err(r.obj_val, f_bf) <= 1e-3
    rp, rd = qpcheck.eps_scaled_residuals(qp, r.x, r.y)
    assert rp <= 1.0 + 1e-9 and rd <= 1.0 + 1e-9
    rt = oracle_lib.solve(qp, eps_abs=1e-10, eps_rel=1e-10, polish=1, max_iter=100000)
    assert rt.status == "solved"
    assert abs(rt.obj_val - f_bf) <= 1e-7 * max(1.0, abs(f_bf))
    assert np.allclose(rt.x, x_bf, atol=1e-5)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", range(5))
def test_diagonal_box_qp_closed_form(oracle_lib, seed):
    """A = I, P = diag(d) > 0: x_i = clip(-q_i/d_i, l_i, u_i), y = -(d x + q)."""
    rng = np.random.default_rng(seed)
    n = 30
    d = rng.uniform(0.1, 10.0, n)
    q = 3 * rng.standard_normal(n)
    l = -rng.random(n)
    u = rng.random(n)
    qp = qpgen.box_qp(d, q, l, u)
    x = np.clip(-q / d, l, u)
    y = -(d * x + q)
    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, max_iter=20000)
    assert r.status == "solved"
    assert np.allclose(r.x, x, atol=1e-6)
    assert np.allclose(r.y, y, atol=1e-6)


def test_box_lp_closed_form(oracle_lib):
    """P = 0, A = I, finite box: x_i = l_i if q_i > 0 else u_i."""
    rng = np.random.default_rng(3)
    n = 20
    q = rng.standard_normal(n)
    l = -rng.random(n) - 0.1
    u = rng.random(n) + 0.1
    qp = qpgen.box_qp(np.zeros(n), q, l, u)
    r = oracle_lib.solve(qp, eps_abs=1e-8, eps_rel=1e-8, max_iter=50000)
    assert r.status == "solved"
    assert np.allclose(r.x, np.where(q > 0, l, u), atol=1e-5)
    assert abs(r.obj_val - q @ np.where(q > 0, l, u)) <= 1e-5


def test_unconstrained_closed_form(oracle_lib):
    """l = -inf, u = +inf: x = -P^-1 q, y = 0."""
    rng = np.random.default_rng(4)
    n, m = 12, 5
    M = rng.standard_normal((n, n))
    P = M @ M.T + np.eye(n)
    q = rng.standard_normal(n)
    A = rng.standard_normal((m, n))
    qp = _qp_dense(P, q, A, -np.inf * np.ones(m), np.inf * np.ones(m))
    r = oracle_lib.solve(qp, eps_abs=1e-10, eps_rel=1e-10, max_iter=20000)
    assert r.status == "solved"
    assert np.allclose(r.x, -np.linalg.solve(P, q), atol=1e-7)
    assert np.allclose(r.y, 0.0, atol=1e-9)


def test_equality_qp_dense_kkt(oracle_lib):
    """Appendix A.2: the solution solves eq. eq_constr_qp_optimality."""
    qp = qpgen.eq_qp(40, qpgen.rng_for(9, 1))
    P, q, A, l, u = qpcheck.dense(qp)
    n, m = P.shape[0], A.shape[0]
    K = np.block([[P, A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-q, l]))
    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, max_iter=50000)
    assert r.status == "solved"
    assert np.allclose(r.x, sol[:n], atol=1e-6)
    assert np.allclose(r.y, sol[n:], atol=1e-5)


@pytest.mark.parametrize("seed", range(3))
def test_equality_qp_is_iterative_refinement(oracle_lib, seed):
    """Appendix A.2: with alpha = 1 and l = u = b, for k >= 1 the ADMM
    iterates (x, y) follow t <- t + (K + dK)^-1 (g - K t), g = (-q, b),
    dK = diag(sigma I, -rho^-1 I), computed here with a dense solve."""
    qp = qpgen.eq_qp(10, qpgen.rng_for(9, 100 + seed))
    P, q, A, b, _ = qpcheck.dense(qp)
    n, m = P.shape[0], A.shape[0]
    sigma, rho_bar = 1e-6, 0.1
    rho = 1e3 * rho_bar * np.ones(m)   # every row is an equality row
    K = np.block([[P, A.T], [A, np.zeros((m, m))]])
    Kt = K + np.diag(np.concatenate([sigma * np.ones(n), -1.0 / rho]))
    g = np.concatenate([-q, b])
    common = dict(alpha=1.0, sigma=sigma, rho=rho_bar, scaling_iters=0, adaptive_rho=0,
                  check_every=10 ** 6, eps_abs=0.0, eps_rel=0.0, polish=0,
                  eps_pinf=0.0, eps_dinf=0.0)
    r1 = oracle_lib.solve(qp, max_iter=1, **common)
    t = np.concatenate([r1.x, r1.y])
    for k in range(2, 7):
        t = t + np.linalg.solve(Kt, g - K @ t)
        rk = oracle_lib.solve(qp, max_iter=k, **common)
        assert rk.status in ("max_iter_reached", "solved")
        assert np.allclose(np.concatenate([rk.x, rk.y]), t, rtol=1e-9, atol=1e-9), k


def test_lasso_zero_above_critical_lambda(oracle_lib):
    """Appendix A.5 with the objective y'y + lam 1't: x = 0 iff
    lam >= 2 ||A'b||_inf; then f = ||b||^2."""
    rng = qpgen.rng_for(9, 7)
    base = qpgen.lasso(rng, 10, 60, density=0.3)
    lam = 2.0 * np.max(np.abs(base.Ad.T @ base.b)) * 1.05
    qp = qpgen.lasso(qpgen.rng_for(9, 7), 10, 60, density=0.3, lam=lam)
    r = oracle_lib.solve(qp, eps_abs=1e-8, eps_rel=1e-8, max_iter=50000, polish=1)
    assert r.status == "solved"
    assert np.max(np.abs(r.x[:10])) <= 1e-6
    assert abs(r.obj_val - base.b @ base.b) <= 1e-6 * (base.b @ base.b)


def test_lasso_orthonormal_soft_threshold(oracle_lib):
    """Orthonormal-column data matrix: x_i = sign(c_i) max(|c_i| - lam/2, 0), c = A'b."""
    rng = np.random.default_rng(11)
    nf, md = 6, 30
    Q, _ = np.linalg.qr(rng.standard_normal((md, nf)))
    b = rng.standard_normal(md)
    c = Q.T @ b
    lam = 0.8 * np.median(np.abs(c)) * 2
    n = nf + md + nf
    Pfull = sp.block_diag([sp.csr_matrix((nf, nf)), 2.0 * sp.identity(md),
                           sp.csr_matrix((nf, nf))]).tocsr()
    qv = np.concatenate([np.zeros(nf + md), lam * np.ones(nf)])
    I = sp.identity(nf)
    A = sp.vstack([sp.hstack([sp.csr_matrix(Q), -sp.identity(md), sp.csr_matrix((md, nf))]),
                   sp.hstack([I, sp.csr_matrix((nf, md)), -I]),
                   sp.hstack([I, sp.csr_matrix((nf, md)), I])]).tocsr()
    l = np.concatenate([b, -np.inf * np.ones(nf), np.zeros(nf)])
    u = np.concatenate([b, np.zeros(nf), np.inf * np.ones(nf)])
    qp = QP(sp.triu(Pfull).tocsr(), qv, A, l, u)
    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, max_iter=100000, polish=1)
    assert r.status == "solved"
    expect = np.sign(c) * np.maximum(np.abs(c) - lam / 2, 0.0)
    assert np.allclose(r.x[:nf], expect, atol=1e-6)


def test_portfolio_without_factors_water_filling(oracle_lib):
    """Appendix A.4 with F = 0: x_i = max(0, (mu_i/gamma - nu)/(2 D_ii)), sum x = 1;
    nu by bisection in FP64."""
    rng = np.random.default_rng(5)
    n, k = 40, 2
    F = sp.csr_matrix((n, k))
    Dd = rng.uniform(0.2, 2.0, n)
    mu = rng.standard_normal(n)
    qp = qpgen.portfolio(rng, model=(F, Dd, mu))
    lo, hi = -100.0, 100.0
    for _ in range(200):
        nu = 0.5 * (lo + hi)
        s = np.maximum(0.0, (mu - nu) / (2 * Dd)).sum()
        lo, hi = (nu, hi) if s > 1 else (lo, nu)
    x = np.maximum(0.0, (mu - nu) / (2 * Dd))
    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, max_iter=100000, polish=1)
    assert r.status == "solved"
    assert np.allclose(r.x[:n], x, atol=1e-6)


def test_mpc_inactive_bounds_is_lqr(oracle_lib):
    """Appendix A.3 with bounds that never bind: the optimum is the
    finite-horizon LQR cost x0' S_0 x0 from the backward Riccati recursion."""
    rng = qpgen.rng_for(9, 3)
    plant = qpgen.mpc_plant(rng, 4, 2)
    Ad, B, Q, R, QT = plant
    x0 = np.array([0.3, -0.2, 0.1, 0.05])
    T = 6
    qp = qpgen.mpc(rng, nx=4, nu=2, T=T, xbar=1e4, ubar=1e4, plant=plant, x_init=x0)
    S = QT.copy()
    for _ in range(T):
        K = np.linalg.solve(R + B.T @ S @ B, B.T @ S @ Ad)
        S = Q + Ad.T @ S @ (Ad - B @ K)
    J = x0 @ S @ x0
    r = oracle_lib.solve(qp, eps_abs=1e-10, eps_rel=1e-10, max_iter=100000, polish=1)
    assert r.status == "solved"
    assert abs(r.obj_val - J) <= 1e-7 * max(1.0, abs(J))


# ---------------------------------------------------------------- infeasibility
def test_primal_infeasible_certificate(oracle_lib):
    """x >= 1 and x <= 0: status primal infeasible and the returned y meets
    the certificate conditions A'y = 0, u'y_+ + l'y_- < 0 (Section 2.1)."""
    qp = _qp_dense([[1.0, 0.0], [0.0, 1.0]], [0.0, 0.0],
                   [[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]],
                   [1.0, -np.inf, -1.0], [np.inf, 0.0, 1.0])
    r = oracle_lib.solve(qp)
    assert r.status == "primal_infeasible"
    y = r.y
    assert np.max(np.abs(qp.A.T @ y)) <= 1e-4 * np.max(np.abs(y))
    yp, ym = np.maximum(y, 0), np.minimum(y, 0)
    supp = sum(qp.u[i] * yp[i] for i in range(3) if yp[i] > 0) + \
        sum(qp.l[i] * ym[i] for i in range(3) if ym[i] < 0)
    assert supp < 0
    assert math.isinf(r.obj_val) and r.obj_val > 0


def test_dual_infeasible_certificate(oracle_lib):
    """P = 0, q = -1, x >= 0: unbounded; the returned x meets Px = 0,
    q'x < 0, (Ax)_i >= 0 on rows with u = +inf (Section 2.1)."""
    n = 5
    qp = qpgen.box_qp(np.zeros(n), -np.ones(n), np.zeros(n), np.inf * np.ones(n))
    r = oracle_lib.solve(qp)
    assert r.status == "dual_infeasible"
    x = r.x
    assert qp.q @ x < 0
    assert np.all(qp.A @ x >= -1e-4 * np.max(np.abs(x)))
    assert math.isinf(r.obj_val) and r.obj_val < 0


def test_max_iter_status(oracle_lib):
    qp = qpgen.config_instance(1, 0)
    r = oracle_lib.solve(qp, max_iter=1)
    assert r.status == "max_iter_reached" and r.iter == 1


# ---------------------------------------------------------------- scaling
def test_scaling_does_not_change_solution(oracle_lib):
    """Section 5.1: the scaled problem has the same solution after unscaling."""
    qp = qpgen.random_qp(30, qpgen.rng_for(9, 21))
    a = oracle_lib.solve(qp, scaling_iters=0, eps_abs=1e-9, eps_rel=1e-9, max_iter=100000)
    b = oracle_lib.solve(qp, scaling_iters=10, eps_abs=1e-9, eps_rel=1e-9, max_iter=100000)
    assert a.status == b.status == "solved"
    assert np.allclose(a.x, b.x, atol=1e-6)
    assert np.allclose(a.y, b.y, atol=1e-5)


def test_ruiz_equilibrates_columns(oracle_lib):
    """With P = 0 and q = 0 the cost step is the identity (gamma = 1) and the
    Ruiz passes drive every column of [0 A'; A 0] to unit infinity norm."""
    rng = np.random.default_rng(2)
    A = qpgen.sparse_normal(rng, 40, 15, 0.3).toarray() * np.exp(3 * rng.standard_normal((40, 1)))
    A[np.abs(A).sum(1) == 0, 0] = 1.0
    A[:, np.abs(A).sum(0) == 0] = 1.0
    qp = _qp_dense(np.zeros((15, 15)), np.zeros(15), A, -np.ones(40), np.ones(40))
    D, E, c = oracle_lib.ruiz(qp, 80)
    Ab = E[:, None] * A * D[None, :]
    assert c == 1.0
    assert np.allclose(np.abs(Ab).max(axis=0), 1.0, atol=1e-6)
    assert np.allclose(np.abs(Ab).max(axis=1), 1.0, atol=1e-6)


def _read_ruiz_golden():
    """Cases of tests/golden/ruiz_passes.txt: (name, qp, [(passes, D, E, c)])."""
    from fractions import Fraction
    cases, cur = [], None
    num = lambda t: float(Fraction(t))  # noqa: E731
    with open(os.path.join(GOLDEN, "ruiz_passes.txt")) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"name": rest.strip(), "passes": []}
                cases.append(cur)
            elif key in ("P", "A"):
                cur[key] = [[num(t) for t in r.split()] for r in rest.split(";")]
            elif key == "q":
                cur["q"] = [num(t) for t in rest.split()]
            elif key == "pass":
                parts = rest.split("|")
                head = parts[0].split()
                cur["passes"].append((int(head[0]), [num(t) for t in head[1:]],
                                      [num(t) for t in parts[1].split()], num(parts[2].strip())))
    out = []
    for c in cases:
        m = len(c["A"])
        qp = _qp_dense(c["P"], c["q"], c["A"], -np.ones(m), np.ones(m), c["name"])
        out.append((c["name"], qp, c["passes"]))
    return out


@pytest.mark.parametrize("case", _read_ruiz_golden(), ids=lambda c: c[0])
def test_ruiz_passes_hand_values(oracle_lib, case):
    """Section 5.1, modified Ruiz equilibration with its cost scaling: D, E
    and c after one and two passes equal the values worked out by hand in
    tests/golden/ruiz_passes.txt (P with an off-diagonal entry, q nonzero; one
    case where the mean column norm of Pbar sets gamma, one where ||qbar||
    does)."""
    name, qp, passes = case
    for k, D_want, E_want, c_want in passes:
        D, E, c = oracle_lib.ruiz(qp, k)
        assert np.allclose(D, D_want, rtol=1e-14, atol=0), (name, k, D, D_want)
        assert np.allclose(E, E_want, rtol=1e-14, atol=0), (name, k, E, E_want)
        assert c == pytest.approx(c_want, rel=1e-14), (name, k, c, c_want)


# ---------------------------------------------------------------- rho-bar rule
def _read_rho_rule():
    rows = []
    with open(os.path.join(GOLDEN, "rho_rule.txt")) as fh:
        for raw in fh:
            t = raw.split("#", 1)[0].split()
            if t:
                rows.append((t[0], *[float(v) for v in t[1:]]))
    return rows


@pytest.mark.parametrize("row", _read_rho_rule(), ids=lambda r: r[0])
def test_rho_rule_hand_values(oracle_lib, row):
    """Section 5.2 rule for rho-bar on synthetic residuals against values
    worked out by hand (tests/golden/rho_rule.txt): the square root of the
    ratio, which normaliser goes with which residual, the 5x gate and its
    boundary, the [1e-6, 1e6] clamp applied before the gate, and the
    zero-normaliser skip."""
    name, rho, pr, pn, dr, dn, want = row
    got = oracle_lib.rho_update(rho, pr, pn, dr, dn)
    assert got == pytest.approx(want, rel=1e-14, abs=0), (name, got, want)


def test_rho_rule_inside_solve_1d(oracle_lib):
    """The Section 5.2 rule as the solver applies it, on a 1-D QP whose first
    ADMM iterate, residuals and normalisers were worked out by hand
    (tests/golden/rho_rule_1d.txt): after the first check rho-bar becomes
    3.1434085266297456."""
    vals = {}
    with open(os.path.join(GOLDEN, "rho_rule_1d.txt")) as fh:
        for raw in fh:
            t = raw.split("#", 1)[0].split()
            if t:
                vals[t[0]] = float(t[1])
    qp = _qp_dense([[vals["P"]]], [vals["q"]], [[vals["A"]]], [vals["l"]], [vals["u"]], "rho1d")
    r = oracle_lib.solve(qp, scaling_iters=0, sigma=vals["sigma"], rho=vals["rho"], alpha=1.0,
                         check_every=1, max_iter=2, adaptive_rho=1, polish=0)
    assert r.rho_updates == int(vals["rho_updates"])
    assert r.rho_bar == pytest.approx(vals["rho_bar_after"], rel=1e-10)


# ---------------------------------------------------------------- invariants
def test_complementarity_invariant(oracle_lib):
    """Section 3.3: for every k >= 1, z = Pi(v) and y = rho (v - Pi(v)) give
    l <= z <= u exactly, y_i > 0 only at z_i = u_i, y_i < 0 only at z_i = l_i."""
    qp = qpgen.random_qp(20, qpgen.rng_for(9, 31))
    for k in (1, 2, 5, 13):
        r = oracle_lib.solve(qp, max_iter=k, scaling_iters=0, check_every=10 ** 6)
        z, y = r.z, r.y
        assert np.all(z >= qp.l) and np.all(z <= qp.u)
        assert np.all(z[y > 0] == qp.u[y > 0])
        assert np.all(z[y < 0] == qp.l[y < 0])


def test_warm_start_from_optimum(oracle_lib):
    """Section 6: warm starting from the solution stops at the first check."""
    qp = qpgen.config_instance(1, 3)
    r = oracle_lib.solve(qp)
    r2 = oracle_lib.solve(qp, x_ws=r.x, y_ws=r.y)
    assert r2.status == "solved" and r2.iter <= 25


@pytest.mark.parametrize("cfg,idx", [(1, 0), (1, 1), (3, 0), (3, 1), (4, 0)])
def test_workload_status_and_acceptance(oracle_lib, cfg, idx):
    """Random QP (x = 0 feasible, P > 0), MPC and portfolio instances solve,
    and the result passes the Section 3.4 test recomputed from (x, y) on the
    original data with z = Pi(Ax)."""
    kw = {"n_range": (100, 400)} if cfg == 4 else {}
    qp = qpgen.config_instance(cfg, idx, **kw)
    r = oracle_lib.solve(qp)
    assert r.status == "solved"
    rp, rd = qpcheck.eps_scaled_residuals(qp, r.x, r.y)
    assert rp <= 1.0 + 1e-6 and rd <= 1.0 + 1e-6
    assert np.isfinite(r.obj_val)


def test_lasso_small_solves(oracle_lib):
    qp = qpgen.lasso(qpgen.rng_for(9, 8), 20, 200, density=0.15)
    r = oracle_lib.solve(qp)
    assert r.status == "solved"
    rp, rd = qpcheck.eps_scaled_residuals(qp, r.x, r.y)
    assert rp <= 1.0 + 1e-6 and rd <= 1.0 + 1e-6


def test_polish_improves_accuracy(oracle_lib):
    """Section 4: a successful polish returns residuals no larger than ADMM's."""
    qp = qpgen.config_instance(4, 0, n_range=(100, 300))
    r0 = oracle_lib.solve(qp, polish=0)
    r1 = oracle_lib.solve(qp, polish=1)
    assert r1.status == "solved"
    if r1.polish_status == 1:
        a0 = qpcheck.acceptance(qp, r0.x, r0.y)
        a1 = qpcheck.acceptance(qp, r1.x, r1.y)
        assert a1[0] <= a0[0] + 1e-12 and a1[1] <= a0[1] + 1e-12
        assert a1[0] <= 1e-8 and a1[1] <= 1e-8


@pytest.mark.parametrize("alpha", [1.0, 1.6, 0.7])
def test_relaxed_contraction_rate_1d(oracle_lib, alpha):
    """1-D unconstrained QP (P = p, A = 1, free row): from x0 = z0 the
    Algorithm 1 iterates keep x = z, y = 0 and, since the KKT step gives
    x~ = ((sigma + rho) x - q) / (p + sigma + rho), the error to x* = -q/p
    contracts by exactly 1 - alpha p / (p + sigma + rho) per iteration."""
    p, q0, sigma, rho = 2.0, -3.0, 1e-6, 0.1
    qp = _qp_dense([[p]], [q0], [[1.0]], [-np.inf], [np.inf])
    xs = -q0 / p
    x0 = 0.25
    rate = 1.0 - alpha * p / (p + sigma + rho)
    for k in (1, 2, 3, 7):
        r = oracle_lib.solve(qp, x_ws=[x0], y_ws=[0.0], max_iter=k, alpha=alpha, sigma=sigma,
                             rho=rho, scaling_iters=0, adaptive_rho=0, check_every=10 ** 6,
                             eps_abs=0.0, eps_rel=0.0, eps_pinf=0.0, eps_dinf=0.0)
        assert abs((r.x[0] - xs) - rate ** k * (x0 - xs)) <= 1e-12
        assert r.z[0] == pytest.approx(r.x[0], abs=1e-14) and r.y[0] == 0.0


@pytest.mark.parametrize("case", _read_golden(), ids=lambda c: c["name"])
def test_polish_recovers_exact_solution(oracle_lib, case):
    """Section 4: from a loose (eps = 1e-3) ADMM solution, polishing with the
    correct active set returns the exact optimum of the hand-solved fixtures."""
    qp = _qp_dense(case["P"], case["q"], case["A"], case["l"], case["u"], case["name"])
    r = oracle_lib.solve(qp, polish=1)
    assert r.status == "solved"
    if r.prim_res == 0.0 and r.dual_res == 0.0:
        pytest.skip("ADMM already exact; nothing for polish to improve")
    assert r.polish_status == 1
    assert np.allclose(r.x, case["x"], atol=1e-9)
    assert abs(r.obj_val - case["f"][0]) <= 1e-9 * max(1.0, abs(case["f"][0]))


def test_polish_matches_brute_force(oracle_lib):
    """Section 4 on the brute-force instances: polishing an eps = 1e-3
    solution must succeed on most of them and, when it does, reproduce the
    enumerated optimum to 1e-8."""
    ok = 0
    for seed in range(40):
        qp = _tiny_random(seed)
        x_bf, _, f_bf = qpcheck.brute_force(qp)
        r = oracle_lib.solve(qp, polish=1)
        assert r.status == "solved"
        if r.polish_status == 1:
            ok += 1
            assert np.allclose(r.x, x_bf, atol=1e-7), seed
            assert abs(r.obj_val - f_bf) <= 1e-8 * max(1.0, abs(f_bf)), seed
    assert ok >= 30


def _equality_with_zero_dual(seed):
    """min 1/2 x'Px + q'x with x_0 = 0 and a slack box on the rest, built so
    that the unconstrained minimiser x* already has x*_0 = 0: x* is the
    solution and the equality row's dual is exactly 0."""
    rng = np.random.default_rng(seed)
    n = 4
    M = rng.standard_normal((n, n))
    P = M @ M.T + 0.5 * np.eye(n)
    xs = rng.standard_normal(n)
    xs[0] = 0.0
    l = -5.0 * np.ones(n)
    u = 5.0 * np.ones(n)
    l[0] = u[0] = 0.0
    qp = QP(sp.csr_matrix(np.triu(P)), -P @ xs, sp.csr_matrix(np.eye(n)), l, u, name=f"eq0 {seed}")
    return qp, xs


def test_polish_accepts_a_sign_free_equality_dual(oracle_lib):
    """Section 4 accepts a polished point that meets the optimality
    conditions.  Here the equality row's dual is 0 at the optimum, so the
    ADMM estimate and the polished value are rounding-sized with either
    sign; a row with l_i = u_i puts no sign condition on its dual, and the
    polished point, the exact optimum, must be accepted on every instance."""
    for seed in range(60):
        qp, xs = _equality_with_zero_dual(seed)
        r = oracle_lib.solve(qp, polish=1)
        assert r.status == "solved" and r.polish_status == 1, seed
        assert np.max(np.abs(r.x - xs)) <= 1e-9 * max(1.0, np.max(np.abs(xs))), seed


@pytest.mark.parametrize("cfg,idx,kw", [(1, 2, {}), (3, 2, {}), (4, 1, {"n_range": (100, 300)}),
                                         (0, 0, {})])
def test_reported_residuals_match_definition(oracle_lib, cfg, idx, kw):
    """The oracle checks in scaled space and unscales (Section 5.1); its
    reported residuals and tolerances must equal the Section 3.4 definitions
    evaluated directly on the original data at the returned (x, z, y)."""
    if cfg == 0:
        # small data: cost scaling gamma > 1, so c != 1 is exercised
        qp = qpgen.random_qp(15, qpgen.rng_for(9, 41))
        qp.P = qp.P * 1e-3
        qp.q = qp.q * 1e-3
    else:
        qp = qpgen.config_instance(cfg, idx, **kw)
    for max_iter in (50, 4000):
        r = oracle_lib.solve(qp, max_iter=max_iter)
        assert r.status in ("solved", "max_iter_reached")
        Pf = qp.full_P()
        Ax, Px, Aty = qp.A @ r.x, Pf @ r.x, qp.A.T @ r.y
        rp = np.max(np.abs(Ax - r.z))
        rd = np.max(np.abs(Px + qp.q + Aty))
        ep = 1e-3 + 1e-3 * max(np.max(np.abs(Ax)), np.max(np.abs(r.z)))
        ed = 1e-3 + 1e-3 * max(np.max(np.abs(Px)), np.max(np.abs(Aty)), np.max(np.abs(qp.q)))
        for a, b in ((r.prim_res, rp), (r.dual_res, rd), (r.eps_prim, ep), (r.eps_dual, ed)):
            assert abs(a - b) <= 1e-9 * max(1.0, abs(b)), (a, b)
    D, E, c = oracle_lib.ruiz(qp, 10)
    if cfg == 0:
        assert c > 2.0


def test_no_false_dual_infeasibility_on_flat_direction(oracle_lib):
    """min 0 s.t. x >= 0 is bounded; from x0 = -1 the iterates move along a
    direction with P dx = 0 and q'dx = 0.  A certificate needs q'dx < 0
    (Section 2.1), so the status must not be dual infeasible."""
    n = 3
    qp = qpgen.box_qp(np.zeros(n), np.zeros(n), np.zeros(n), np.inf * np.ones(n))
    # at k = 24 the step dx is positive in every coordinate, so every other
    # condition of the dual test holds there
    r = oracle_lib.solve(qp, x_ws=-np.ones(n), y_ws=np.zeros(n), max_iter=24,
                         eps_abs=1e-14, eps_rel=1e-14, scaling_iters=0)
    assert r.status == "max_iter_reached"
    assert np.all(r.x > 0.6)


def test_no_false_primal_infeasibility_on_duplicate_equalities(oracle_lib):
    """Two copies of the row x = 1: feasible.  A dual split dy = (t, -t) has
    A'dy = 0 and u'dy_+ + l'dy_- = 0; a certificate needs the latter < 0."""
    qp = _qp_dense([[0.0]], [-1.0], [[1.0], [1.0]], [1.0, 1.0], [1.0, 1.0])
    r = oracle_lib.solve(qp, x_ws=[1.0], y_ws=[3.0, -2.0], max_iter=25, eps_abs=1e-14,
                         eps_rel=1e-14, scaling_iters=0, adaptive_rho=0)
    assert r.status != "primal_infeasible"


# ------------------------------------------- appendix fitting problems, restated
def test_huber_qp_equals_huber_loss_minimum(oracle_lib):
    """Appendix Huber fitting: eliminating (u, r, s) from the QP leaves the sum
    of Huber penalties of the residuals Ax - b (quadratic inside M, linear with
    slope 2M outside).  That smooth unconstrained problem is minimised here by
    scipy's L-BFGS on the data block alone; the oracle's optimal objective and
    x-part must match it."""
    from scipy.optimize import minimize
    nf, md, M = 6, 120, 1.0
    qp = qpgen.huber(qpgen.rng_for(7, 31), nf, m_data=md, M=M)
    Ad = qp.A[:md, :nf].toarray()
    b = qp.l[:md]

    def f(x):
        e = Ad @ x - b
        a = np.abs(e)
        val = np.where(a <= M, e * e, 2.0 * M * a - M * M).sum()
        g = Ad.T @ np.where(a <= M, 2.0 * e, 2.0 * M * np.sign(e))
        return val, g

    ref = minimize(f, np.zeros(nf), jac=True, method="L-BFGS-B",
                   options={"ftol": 1e-15, "gtol": 1e-11, "maxiter": 10000})
    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, max_iter=200000, polish=1)
    assert r.status == "solved"
    assert abs(r.obj_val - ref.fun) <= 1e-7 * max(1.0, abs(ref.fun)), (r.obj_val, ref.fun)
    assert np.allclose(r.x[:nf], ref.x, atol=1e-5)


def test_svm_qp_equals_hinge_loss_minimum(oracle_lib):
    """Appendix SVM: with t eliminated the QP is x'x + lam sum max(0, 1 + b_i a_i'x),
    i.e. half of it is the soft-margin linear SVM 0.5 w'w + C sum hinge(y_i a_i'w)
    with C = lam / 2 and labels y = -b, without an intercept.  scikit-learn's
    liblinear (dual coordinate descent) solves that; its optimum, doubled, must
    equal the oracle's objective, and the weights must agree."""
    from sklearn.svm import LinearSVC
    nf, md, lam = 5, 200, 1.0
    qp = qpgen.svm(qpgen.rng_for(7, 41), nf, m_data=md, lam=lam)
    Ab = -qp.A[:md, :nf].toarray()            # rows b_i a_i'
    b = np.where(np.arange(md) < md // 2, 1.0, -1.0)
    Ad = Ab * b[:, None]
    clf = LinearSVC(C=lam / 2.0, loss="hinge", dual=True, fit_intercept=False,
                    tol=1e-12, max_iter=1000000)
    clf.fit(Ad, -b)
    w = clf.coef_.ravel()

    def obj(x):
        return x @ x + lam * np.maximum(0.0, 1.0 + Ab @ x).sum()

    r = oracle_lib.solve(qp, eps_abs=1e-9, eps_rel=1e-9, max_iter=200000, polish=1)
    assert r.status == "solved"
    f_ref = obj(w)
    assert abs(r.obj_val - f_ref) <= 1e-6 * max(1.0, abs(f_ref)), (r.obj_val, f_ref)
    assert abs(obj(r.x[:nf]) - r.obj_val) <= 1e-7 * max(1.0, abs(f_ref))
    assert np.allclose(r.x[:nf], w, atol=1e-4)
