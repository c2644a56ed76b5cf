"""Independent numpy checks used by the tests (no oracle, no GPU code).

* brute-force active-set enumeration of the KKT conditions (Section 2,
  eqs. prim_feas, dual_feas, compl_slack) for tiny strictly convex QPs;
* the solver-independent acceptance test of Section 8 (z-free primal
  residual and dual residual, unscaled);
* the termination criterion of Section 3.4 with z = projection of Ax.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def dense(qp):
    P = qp.full_P().toarray()
    A = qp.A.toarray()
    return P, qp.q.copy(), A, qp.l.copy(), qp.u.copy()


def brute_force(qp, tol=1e-9):
    """Optimal (x, y, f) of a tiny QP with P > 0 by enumerating every
    assignment of each row to {inactive, at lower, at upper} and solving the
    equality-constrained KKT system; keeps candidates that are primal
    feasible and have duals of the right sign (y <= 0 at l, y >= 0 at u)."""
    P, q, A, l, u = dense(qp)
    n, m = P.shape[0], A.shape[0]
    best = None
    choices = []
    for i in range(m):
        c = [0]
        if np.isfinite(l[i]):
            c.append(-1)
        if np.isfinite(u[i]) and not (l[i] == u[i]):
            c.append(1)
        if l[i] == u[i]:
            c = [-1]   # equality row: always active
        choices.append(c)
    for assign in itertools.product(*choices):
        W = [i for i in range(m) if assign[i] != 0]
        bW = np.array([l[i] if assign[i] < 0 else u[i] for i in W])
        k = len(W)
        K = np.zeros((n + k, n + k))
        K[:n, :n] = P
        if k:
            K[:n, n:] = A[W].T
            K[n:, :n] = A[W]
        rhs = np.concatenate([-q, bW])
        # least squares: degenerate active sets (dependent rows) still have
        # a consistent solution whose x is unique when P > 0
        sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
        if not np.allclose(K @ sol, rhs, atol=1e-9, rtol=1e-9):
            continue
        x = sol[:n]
        y = np.zeros(m)
        y[W] = sol[n:]
        Ax = A @ x
        if np.any(Ax < l - tol) or np.any(Ax > u + tol):
            continue
        ok = True
        for i in W:
            if l[i] == u[i]:
                continue
            if assign[i] < 0 and y[i] > tol:
                ok = False
            if assign[i] > 0 and y[i] < -tol:
                ok = False
        if not ok:
            continue
        f = 0.5 * x @ P @ x + q @ x
        if best is None or f < best[2]:
            best = (x, y, f)
    return best


def acceptance(qp, x, y):
    """Section 8 acceptance quantities on the original data:
    zfree_prim = ||(Ax - u)_+ + (Ax - l)_-||_inf, dual = ||Px + q + A'y||_inf."""
    Pf = qp.full_P()
    Ax = qp.A @ x
    viol = np.maximum(Ax - qp.u, 0.0) + np.minimum(Ax - qp.l, 0.0)
    rd = Pf @ x + qp.q + qp.A.T @ y
    return float(np.max(np.abs(viol), initial=0.0)), float(np.max(np.abs(rd), initial=0.0))


def eps_scaled_residuals(qp, x, y, eps_abs=1e-3, eps_rel=1e-3):
    """r_prim / eps_prim and r_dual / eps_dual of Section 3.4 on the original
    data, with z the projection of Ax onto [l, u] (so r_prim is z-free)."""
    Pf = qp.full_P()
    Ax = qp.A @ x
    z = np.minimum(np.maximum(Ax, qp.l), qp.u)
    Px = Pf @ x
    Aty = qp.A.T @ y
    rp = np.max(np.abs(Ax - z), initial=0.0)
    rd = np.max(np.abs(Px + qp.q + Aty), initial=0.0)
    ep = eps_abs + eps_rel * max(np.max(np.abs(Ax), initial=0.0), np.max(np.abs(z), initial=0.0))
    ed = eps_abs + eps_rel * max(np.max(np.abs(Px), initial=0.0),
                                 np.max(np.abs(Aty), initial=0.0),
                                 np.max(np.abs(qp.q), initial=0.0))
    return float(rp / ep), float(rd / ed)


def rel_obj_err(f, f_ref):
    return abs(f - f_ref) / max(1.0, abs(f_ref))


def kkt_upper(P, A, sigma, rho):
    """Upper triangle (CSC) of the ADMM KKT matrix, for LDL tests."""
    n = P.shape[0]
    m = A.shape[0]
    K = sp.bmat([[sp.csr_matrix(P) + sigma * sp.identity(n), sp.csr_matrix(A).T],
                 [sp.csr_matrix(A), -sp.diags(1.0 / rho)]])
    return sp.triu(K).tocsc(), K.toarray()
