"""Seeded synthetic QP generators.

This module only builds problem data (P, q, A, l, u) for the workload classes of
the paper's appendix; it holds none of the solver's arithmetic.  It is shared
by the tests, the benchmark and the oracle's checks.  Every generator draws from
``numpy.random.default_rng(SeedSequence([cfg, index]))`` so that a (cfg, index)
pair always names the same instance.

Conventions:

* Matrices are returned as ``scipy.sparse.csr_matrix`` with float64 values and
  sorted column indices; ``P`` is the upper triangle (diagonal included).
* Infinite bounds are IEEE ``inf``.
* "p% density" means every entry is nonzero independently with probability p,
  value N(0,1) unless stated otherwise.
* ``N(mu, v)`` takes the variance as second argument.
* The paper's objectives without a 1/2 factor are written as P = 2*(...).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "QP", "rng_for", "sparse_normal", "random_qp", "eq_qp", "lasso",
    "mpc", "portfolio", "huber", "banded", "few_dense_rows", "box_qp", "config_instance",
    "serving_trace",
]


@dataclasses.dataclass
class QP:
    """A QP  min 1/2 x'Px + q'x  s.t.  l <= Ax <= u  (P given as its upper triangle)."""

    P: sp.csr_matrix          # n x n upper triangle, float64
    q: np.ndarray             # n
    A: sp.csr_matrix          # m x n, float64
    l: np.ndarray             # m (may hold -inf)
    u: np.ndarray             # m (may hold +inf)
    name: str = ""

    @property
    def n(self) -> int:
        return self.P.shape[0]

    @property
    def m(self) -> int:
        return self.A.shape[0]

    def full_P(self) -> sp.csr_matrix:
        """Symmetric P from its upper triangle (diagonal counted once)."""
        U = self.P.tocsr()
        D = sp.diags(U.diagonal())
        return (U + U.T - D).tocsr()

    def objective(self, x: np.ndarray) -> float:
        Px = self.full_P() @ x
        return float(0.5 * x @ Px + self.q @ x)


def rng_for(cfg: int, index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(index)]))


def _csr(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M, dtype=np.float64)
    M.sum_duplicates()
    M.sort_indices()
    M.eliminate_zeros()
    return M


def sparse_normal(rng: np.random.Generator, rows: int, cols: int, density: float,
                  scale: float = 1.0, mean: float = 0.0,
                  chunk_cells: int = 1 << 24) -> sp.csr_matrix:
    """rows x cols matrix, each entry nonzero with probability `density`,
    nonzero values ~ N(mean, scale^2).  Drawn row-block by row-block so that
    memory stays bounded for large instances."""
    indptr = [np.zeros(1, dtype=np.int64)]
    idx_parts, val_parts = [], []
    rows_per_chunk = max(1, chunk_cells // max(cols, 1))
    nnz_so_far = 0
    for r0 in range(0, rows, rows_per_chunk):
        r1 = min(rows, r0 + rows_per_chunk)
        mask = rng.random((r1 - r0, cols)) < density
        rr, cc = np.nonzero(mask)
        vals = mean + scale * rng.standard_normal(rr.size)
        counts = np.bincount(rr, minlength=r1 - r0)
        indptr.append(nnz_so_far + np.cumsum(counts))
        nnz_so_far += rr.size
        idx_parts.append(cc.astype(np.int32))
        val_parts.append(vals)
    indptr = np.concatenate(indptr).astype(np.int64)
    idx = np.concatenate(idx_parts) if idx_parts else np.zeros(0, np.int32)
    val = np.concatenate(val_parts) if val_parts else np.zeros(0)
    M = sp.csr_matrix((val, idx, indptr), shape=(rows, cols))
    M.sort_indices()
    return M


def _upper(Pfull) -> sp.csr_matrix:
    return _csr(sp.triu(sp.csr_matrix(Pfull)))


# --------------------------------------------------------------------------
# Appendix A.1: random QP
# --------------------------------------------------------------------------
def random_qp(n: int, rng: np.random.Generator, m: int | None = None,
              density: float = 0.15) -> QP:
    """P = M M' + 1e-2 I with M n x n at `density`; A m x n (m = 10n) at
    `density`; q ~ N(0,1); l = -U[0,1]; u = U[0,1]."""
    m = 10 * n if m is None else m
    M = sparse_normal(rng, n, n, density)
    Pfull = (M @ M.T) + 1e-2 * sp.identity(n)
    A = sparse_normal(rng, m, n, density)
    q = rng.standard_normal(n)
    l = -rng.random(m)
    u = rng.random(m)
    return QP(_upper(Pfull), q, _csr(A), l, u, name=f"random_qp(n={n},m={m})")


# --------------------------------------------------------------------------
# Appendix A.2: equality-constrained QP
# --------------------------------------------------------------------------
def eq_qp(n: int, rng: np.random.Generator, density: float = 0.15) -> QP:
    m = n // 2
    M = sparse_normal(rng, n, n, density)
    Pfull = (M @ M.T) + 1e-2 * sp.identity(n)
    A = sparse_normal(rng, m, n, density)
    q = rng.standard_normal(n)
    b = rng.standard_normal(m)
    return QP(_upper(Pfull), q, _csr(A), b.copy(), b.copy(), name=f"eq_qp(n={n})")


# --------------------------------------------------------------------------
# Appendix A.3: optimal control (MPC), with the batched-MPC workload's changes
# --------------------------------------------------------------------------
def _dare(Ad: np.ndarray, B: np.ndarray, Q: np.ndarray, R: np.ndarray,
          tol: float = 1e-12, max_iter: int = 100000) -> np.ndarray:
    """Stabilising solution of the discrete algebraic Riccati equation by
    fixed-point (value) iteration; converges for stable Ad."""
    X = Q.copy()
    for _ in range(max_iter):
        BtX = B.T @ X
        K = np.linalg.solve(R + BtX @ B, BtX @ Ad)
        Xn = Q + Ad.T @ X @ Ad - Ad.T @ X @ B @ K
        Xn = 0.5 * (Xn + Xn.T)
        if np.max(np.abs(Xn - X)) <= tol * max(1.0, np.max(np.abs(Xn))):
            return Xn
        X = Xn
    raise RuntimeError("DARE fixed-point iteration did not converge")


def mpc_plant(rng: np.random.Generator, nx: int = 20, nu: int = 10,
              dyn_var: float = 0.1, spectral_radius: float = 0.98):
    """Dynamics, costs and terminal cost of one plant."""
    Ad = np.eye(nx) + math.sqrt(dyn_var) * rng.standard_normal((nx, nx))
    rad = np.max(np.abs(np.linalg.eigvals(Ad)))
    Ad = Ad * (spectral_radius / rad)
    B = rng.standard_normal((nx, nu))
    Q = np.diag(10.0 * rng.random(nx))
    R = 0.1 * np.eye(nu)
    QT = _dare(Ad, B, Q, R)
    return Ad, B, Q, R, QT


def mpc(rng: np.random.Generator, nx: int = 20, nu: int = 10, T: int | None = None,
        T_range=(5, 20), xbar: float = 5.0, ubar: float = 1.0,
        plant=None, x_init: np.ndarray | None = None) -> QP:
    """Variables (x_0..x_T, u_0..u_{T-1}); rows: x_0 = x_init, dynamics
    x_{t+1} - Ad x_t - B u_t = 0, then box rows on every variable.
    Cost x_T'Q_T x_T + sum x_t'Qx_t + u_t'Ru_t, i.e. P = 2 blkdiag(Q..Q, Q_T, R..R)."""
    if T is None:
        T = int(rng.integers(T_range[0], T_range[1] + 1))
    if plant is None:
        plant = mpc_plant(rng, nx, nu)
    Ad, B, Q, R, QT = plant
    if x_init is None:
        x_init = rng.uniform(-1.0, 1.0, nx)
    nX = nx * (T + 1)
    n = nX + nu * T
    blocks = [Q] * T + [QT] + [R] * T
    Pfull = 2.0 * sp.block_diag(blocks, format="csr")
    q = np.zeros(n)
    rows = []
    # initial state
    rows.append(sp.hstack([sp.identity(nx), sp.csr_matrix((nx, n - nx))]))
    # dynamics: -Ad x_t + x_{t+1} - B u_t = 0
    Sx = sp.kron(sp.eye(T, T + 1, k=1), sp.identity(nx)) + sp.kron(sp.eye(T, T + 1), -Ad)
    Su = sp.kron(sp.identity(T), -B)
    rows.append(sp.hstack([Sx, Su]))
    rows.append(sp.identity(n))
    A = _csr(sp.vstack(rows))
    l = np.concatenate([x_init, np.zeros(nx * T), -xbar * np.ones(nX), -ubar * np.ones(nu * T)])
    u = np.concatenate([x_init, np.zeros(nx * T), xbar * np.ones(nX), ubar * np.ones(nu * T)])
    return QP(_upper(Pfull), q, A, l, u, name=f"mpc(nx={nx},nu={nu},T={T})")


# --------------------------------------------------------------------------
# Appendix A.4: factor-model portfolio
# --------------------------------------------------------------------------
def portfolio_model(rng: np.random.Generator, n: int, k: int | None = None,
                    density: float = 0.5):
    k = max(1, n // 10) if k is None else k
    F = sparse_normal(rng, n, k, density)
    Dd = rng.uniform(0.0, math.sqrt(k), n)
    mu = rng.standard_normal(n)
    return F, Dd, mu


def portfolio(rng: np.random.Generator, n: int | None = None, n_range=(100, 2000),
              gamma: float = 1.0, model=None) -> QP:
    """Variables (x in R^n, y in R^k); min x'Dx + y'y - mu'x/gamma
    s.t. y = F'x, 1'x = 1, x >= 0."""
    if model is None:
        if n is None:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
        model = portfolio_model(rng, n)
    F, Dd, mu = model
    n, k = F.shape
    Pfull = 2.0 * sp.diags(np.concatenate([Dd, np.ones(k)]))
    q = np.concatenate([-mu / gamma, np.zeros(k)])
    A = sp.vstack([
        sp.hstack([F.T, -sp.identity(k)]),
        sp.hstack([sp.csr_matrix(np.ones((1, n))), sp.csr_matrix((1, k))]),
        sp.hstack([sp.identity(n), sp.csr_matrix((n, k))]),
    ])
    l = np.concatenate([np.zeros(k), [1.0], np.zeros(n)])
    u = np.concatenate([np.zeros(k), [1.0], np.full(n, np.inf)])
    return QP(_upper(Pfull), q, _csr(A), l, u, name=f"portfolio(n={n},k={k})")


# --------------------------------------------------------------------------
# Appendix A.5: Lasso
# --------------------------------------------------------------------------
def lasso(rng: np.random.Generator, n_features: int, m_data: int | None = None,
          density: float = 0.15, lam_frac: float = 0.2, lam: float | None = None) -> QP:
    """Variables (x, y, t); min y'y + lam 1't  s.t.  y = Ad x - b,  -t <= x <= t."""
    nf = n_features
    md = 100 * nf if m_data is None else m_data
    Ad = sparse_normal(rng, md, nf, density)
    v = np.where(rng.random(nf) < 0.5, 0.0, rng.standard_normal(nf) / math.sqrt(nf))
    b = Ad @ v + rng.standard_normal(md)
    if lam is None:
        lam = lam_frac * np.max(np.abs(Ad.T @ b))
    n = nf + md + nf
    Pfull = sp.block_diag([sp.csr_matrix((nf, nf)), 2.0 * sp.identity(md),
                           sp.csr_matrix((nf, nf))], format="csr")
    q = np.concatenate([np.zeros(nf + md), lam * np.ones(nf)])
    I = sp.identity(nf)
    A = sp.vstack([
        sp.hstack([Ad, -sp.identity(md), sp.csr_matrix((md, nf))]),
        sp.hstack([I, sp.csr_matrix((nf, md)), -I]),
        sp.hstack([I, sp.csr_matrix((nf, md)), I]),
    ])
    l = np.concatenate([b, -np.inf * np.ones(nf), np.zeros(nf)])
    u = np.concatenate([b, np.zeros(nf), np.inf * np.ones(nf)])
    qp = QP(_upper(Pfull), q, _csr(A), l, u, name=f"lasso(nf={nf},md={md})")
    qp.Ad, qp.b, qp.lam = Ad, b, lam  # kept for closed-form checks
    return qp


# --------------------------------------------------------------------------
# Appendix A.6: Huber fitting
# --------------------------------------------------------------------------
def huber(rng: np.random.Generator, n_features: int, m_data: int | None = None,
          density: float = 0.15, M: float = 1.0) -> QP:
    """Variables (x, u, r, s); min u'u + 2M 1'(r+s)  s.t. Ax - b - u = r - s, r,s >= 0."""
    nf = n_features
    md = 100 * nf if m_data is None else m_data
    Ad = sparse_normal(rng, md, nf, density)
    v = rng.standard_normal(nf) / math.sqrt(nf)
    out = rng.random(md) < 0.05
    eps = np.where(out, rng.uniform(0.0, 10.0, md), 0.5 * rng.standard_normal(md))
    b = Ad @ v + eps
    n = nf + 3 * md
    Pfull = sp.block_diag([sp.csr_matrix((nf, nf)), 2.0 * sp.identity(md),
                           sp.csr_matrix((2 * md, 2 * md))], format="csr")
    q = np.concatenate([np.zeros(nf + md), 2.0 * M * np.ones(2 * md)])
    Im = sp.identity(md)
    A = sp.vstack([
        sp.hstack([Ad, -Im, -Im, Im]),
        sp.hstack([sp.csr_matrix((2 * md, nf + md)), sp.identity(2 * md)]),
    ])
    l = np.concatenate([b, np.zeros(2 * md)])
    u = np.concatenate([b, np.inf * np.ones(2 * md)])
    return QP(_upper(Pfull), q, _csr(A), l, u, name=f"huber(nf={nf},md={md})")


# --------------------------------------------------------------------------
# A banded structure of a chosen half-bandwidth (edge cases of the band factor)
# --------------------------------------------------------------------------
def banded(rng: np.random.Generator, n: int, w: int, stride: int = 8) -> QP:
    """A QP whose reduced matrix P + A'RA has half-bandwidth exactly w in the
    natural order: P tridiagonal (diagonal U[1, 2], off-diagonal U[-0.3,
    0.3]), rows of A over the windows of w + 1 consecutive variables starting
    every `stride`-th variable (entries N(0, 1/(w+1)), bounds [-0.5, 0.5]),
    then a box [-1, 1] on every variable; q ~ N(0, 4)."""
    main = rng.uniform(1.0, 2.0, n)
    off = rng.uniform(-0.3, 0.3, n - 1)
    P = sp.diags([main, off], [0, 1], format="csr")
    starts = np.arange(0, n - w, stride)
    rows = np.repeat(np.arange(len(starts)), w + 1)
    cols = (starts[:, None] + np.arange(w + 1)[None, :]).ravel()
    vals = rng.standard_normal(len(cols)) / math.sqrt(w + 1)
    W = sp.csr_matrix((vals, (rows, cols)), shape=(len(starts), n))
    A = sp.vstack([W, sp.identity(n)], format="csr")
    l = np.concatenate([-0.5 * np.ones(len(starts)), -np.ones(n)])
    u = np.concatenate([0.5 * np.ones(len(starts)), np.ones(n)])
    q = 2.0 * rng.standard_normal(n)
    return QP(_csr(P), q, _csr(A), l, u, name=f"banded(n={n},w={w})")


def few_dense_rows(rng: np.random.Generator, n: int, rows: int = 6, box: float = 2.0) -> QP:
    """A large QP whose reduced matrix is dense but cheap to factor exactly
    on the CPU: P tridiagonal (diagonal U[1, 2], off-diagonal U[-0.3, 0.3]),
    `rows` dense rows of A (entries N(0, 1/n), bounds [-0.1, 0.1]) and a box
    [-box, box] on every variable; q ~ N(0, 9)."""
    P = sp.diags([rng.uniform(1.0, 2.0, n), rng.uniform(-0.3, 0.3, n - 1)], [0, 1], format="csr")
    W = rng.standard_normal((rows, n)) / math.sqrt(n)
    A = sp.vstack([sp.csr_matrix(W), sp.identity(n)], format="csr")
    l = np.concatenate([-0.1 * np.ones(rows), -box * np.ones(n)])
    u = np.concatenate([0.1 * np.ones(rows), box * np.ones(n)])
    return QP(_csr(P), 3.0 * rng.standard_normal(n), _csr(A), l, u,
              name=f"few_dense_rows(n={n},rows={rows})")


# --------------------------------------------------------------------------
# Small structured instances used by the closed-form checks
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# Appendix A.7: support vector machine
# --------------------------------------------------------------------------
def svm(rng: np.random.Generator, n_features: int, m_data: int | None = None,
        density: float = 0.15, lam: float = 1.0) -> QP:
    """Variables (x, t); min x'x + lam 1't  s.t.  t >= diag(b) A x + 1, t >= 0.
    b = +1 on the first m/2 points, -1 on the rest; the entries of A are
    N(+1/n, 1/n) on the first half and N(-1/n, 1/n) on the second, 15% dense.
    Readings (not stated in the appendix): m = 100 n as for the other fitting
    problems, lam = 1."""
    nf = n_features
    md = 100 * nf if m_data is None else m_data
    half = md // 2
    mask = rng.random((md, nf)) < density
    mean = np.where(np.arange(md)[:, None] < half, 1.0 / nf, -1.0 / nf)
    vals = mean + math.sqrt(1.0 / nf) * rng.standard_normal((md, nf))
    Ad = sp.csr_matrix(np.where(mask, vals, 0.0))
    b = np.where(np.arange(md) < half, 1.0, -1.0)
    n = nf + md
    Pfull = sp.block_diag([2.0 * sp.identity(nf), sp.csr_matrix((md, md))], format="csr")
    q = np.concatenate([np.zeros(nf), lam * np.ones(md)])
    A = sp.vstack([
        sp.hstack([-sp.diags(b) @ Ad, sp.identity(md)]),
        sp.hstack([sp.csr_matrix((md, nf)), sp.identity(md)]),
    ])
    l = np.concatenate([np.ones(md), np.zeros(md)])
    u = np.full(2 * md, np.inf)
    return QP(_upper(Pfull), q, _csr(A), l, u, name=f"svm(nf={nf},md={md})")


def box_qp(d: np.ndarray, q: np.ndarray, l: np.ndarray, u: np.ndarray) -> QP:
    """min 1/2 x'diag(d)x + q'x  s.t.  l <= x <= u  (A = I)."""
    n = d.size
    return QP(_csr(sp.diags(d)), np.asarray(q, float), _csr(sp.identity(n)),
              np.asarray(l, float), np.asarray(u, float), name=f"box_qp(n={n})")


# --------------------------------------------------------------------------
# The five named workloads
# --------------------------------------------------------------------------
def config_instance(cfg: int, index: int = 0, **overrides) -> QP:
    """Instance `index` of workload `cfg`:
    1 random QP n=50, m=500;  2 Lasso 10000x2000 at 5%;  3 MPC nx=20, nu=10,
    T in {5..20};  4 portfolio n in {100..2000}, k = n/10."""
    rng = rng_for(cfg, index)
    if cfg == 1:
        return random_qp(overrides.get("n", 50), rng, m=overrides.get("m", None))
    if cfg == 2:
        return lasso(rng, overrides.get("n_features", 2000),
                     overrides.get("m_data", 10000), density=overrides.get("density", 0.05))
    if cfg == 3:
        return mpc(rng, T=overrides.get("T", None))
    if cfg == 4:
        return portfolio(rng, n=overrides.get("n", None),
                         n_range=overrides.get("n_range", (100, 2000)))
    raise ValueError(f"unknown workload {cfg}")


def serving_trace(n_requests: int, rate: float, seed_index: int = 0,
                  n_range=(20, 5000), n_plants: int = 64, n_models: int = 16):
    """Poisson arrival trace for the serving workload.

    Returns a list of dicts {t, kind, key, index} where kind is 'random',
    'mpc' or 'portfolio' (one third each), `key` names the structure a
    repeated request shares (None for fresh random QPs) and `index` seeds the
    instance.  The problem data for a request is built by `serving_request`."""
    rng = rng_for(5, seed_index)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps)
    kinds = rng.integers(0, 3, n_requests)
    out = []
    for i in range(n_requests):
        kind = ("random", "mpc", "portfolio")[int(kinds[i])]
        if kind == "random":
            key = None
        elif kind == "mpc":
            key = ("mpc", int(rng.integers(0, n_plants)))
        else:
            key = ("portfolio", int(rng.integers(0, n_models)))
        out.append(dict(t=float(t[i]), kind=kind, key=key, index=i + 1))
    return out


def serving_request(req: dict, state: dict, n_range=(20, 5000)) -> QP:
    """Problem data for one trace entry.  Repeats of an MPC plant change only
    x_init (l, u); repeats of a portfolio model update mu <- 0.9 mu + N(0, 0.1)
    (q only).  `state` carries the per-key models across calls."""
    rng = rng_for(5, req["index"])
    if req["kind"] == "random":
        lo, hi = math.log(n_range[0]), math.log(n_range[1])
        n = int(round(math.exp(rng.uniform(lo, hi))))
        return random_qp(n, rng)
    key = req["key"]
    if req["kind"] == "mpc":
        if key not in state:
            prng = rng_for(50, key[1])
            plant = mpc_plant(prng)
            T = int(prng.integers(5, 21))
            state[key] = (plant, T)
        plant, T = state[key]
        return mpc(rng, T=T, plant=plant)
    if key not in state:
        prng = rng_for(51, key[1])
        state[key] = list(portfolio_model(prng, int(prng.integers(100, 2001))))
    F, Dd, mu = state[key]
    mu = 0.9 * mu + math.sqrt(0.1) * rng.standard_normal(mu.size)
    state[key][2] = mu
    return portfolio(rng, model=(F, Dd, mu))
