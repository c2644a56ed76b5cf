"""GPU parity against the FP64 CPU oracle, through the C ABI (the ctypes
binding only marshals arguments).  Statuses must match exactly; solved
results must pass the Section 3.4 test recomputed in FP64 on the original
data, and the objective must agree to 1e-3 relative."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import qpgen
from qpgen import QP
from tests import gpu_common as gc
from tests import qpcheck

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    assert pm.device_count() > 0, "no HIP device"
    return pm


def _solve_batch(pm, qps, **settings):
    b = pm.Batch(qps, **settings)
    b.solve()
    res = [b.get(i) for i in range(len(qps))]
    b.close()
    return res


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_random_qp_single_instance(pm, precision):
    """Workload 1 (random QP, n=50, m=500) as single instances."""
    rows = []
    for i in range(3):
        qp = qpgen.config_instance(1, i)
        print(f"random_qp seed [1,{i}] {precision}", flush=True)
        x, y, info = pm.solve(qp, precision=precision)
        rows.append(gc.compare(qp, x, y, info, oracle.solve(qp)))
    errs = gc.summarize(rows, f"random_qp single {precision}")
    assert max(errs) <= gc.OBJ_TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_random_qp_100_seeds(pm, precision):
    """Workload 1 over seeds [1,0..99], solved as one batch."""
    qps = [qpgen.config_instance(1, i) for i in range(100)]
    print(f"random_qp 100 seeds {precision}", flush=True)
    res = _solve_batch(pm, qps, precision=precision)
    rows = [gc.compare(qp, *r, oracle.solve(qp)) for qp, r in zip(qps, res)]
    gc.summarize(rows, f"random_qp x100 {precision}")
    gc.assert_obj_parity(rows, f"random_qp x100 {precision}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_mpc_batch(pm, precision):
    """Workload 3 generator (MPC, T in 5..20), 96 instances, 24 checked."""
    qps = [qpgen.config_instance(3, i) for i in range(96)]
    print(f"mpc x96 {precision}", flush=True)
    res = _solve_batch(pm, qps, precision=precision)
    rows = [gc.compare(qps[i], *res[i], oracle.solve(qps[i])) for i in range(0, 96, 4)]
    gc.summarize(rows, f"mpc x96 {precision}")
    gc.assert_obj_parity(rows, f"mpc x96 {precision}")


def test_portfolio_batch_status_and_residuals(pm):
    """Workload 4 generator (portfolio), 12 instances with n in 100..800,
    unpolished: status, eps-scaled residuals and objective."""
    qps = [qpgen.config_instance(4, i, n_range=(100, 800)) for i in range(12)]
    print("portfolio x12 fp32", flush=True)
    res = _solve_batch(pm, qps, precision="fp32")
    rows = [gc.compare(qps[i], *res[i], oracle.solve(qps[i])) for i in range(12)]
    gc.summarize(rows, "portfolio x12 fp32 (unpolished)")
    gc.assert_obj_parity(rows, "portfolio x12 fp32 (unpolished)")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_lasso_small(pm, precision):
    qp = qpgen.lasso(qpgen.rng_for(9, 5), 50, 500, density=0.15)
    print(f"lasso 50x500 {precision}", flush=True)
    x, y, info = pm.solve(qp, precision=precision)
    row = gc.compare(qp, x, y, info, oracle.solve(qp))
    assert row["obj_err"] <= gc.OBJ_TOL


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_primal_infeasible(pm, precision):
    A = sp.csr_matrix(np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
    qp = QP(sp.csr_matrix(np.eye(2)), np.zeros(2), A, np.array([1.0, -np.inf, -1.0]),
            np.array([np.inf, 0.0, 1.0]))
    print(f"primal infeasible {precision}", flush=True)
    x, y, info = pm.solve(qp, precision=precision)
    assert info["status_name"] == "primal_infeasible"
    assert np.max(np.abs(A.T @ y)) <= 1e-3 * np.max(np.abs(y))
    supp = sum(qp.u[i] * y[i] for i in range(3) if y[i] > 0) + \
        sum(qp.l[i] * y[i] for i in range(3) if y[i] < 0)
    assert supp < 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_dual_infeasible(pm, precision):
    n = 5
    qp = qpgen.box_qp(np.zeros(n), -np.ones(n), np.zeros(n), np.inf * np.ones(n))
    print(f"dual infeasible {precision}", flush=True)
    x, y, info = pm.solve(qp, precision=precision)
    assert info["status_name"] == "dual_infeasible"
    assert qp.q @ x < 0
    assert np.all(qp.A @ x >= -1e-3 * np.max(np.abs(x)))


def test_max_iter_status(pm):
    qp = qpgen.config_instance(1, 0)
    x, y, info = pm.solve(qp, max_iter=1)
    assert info["status_name"] == "max_iter_reached" and info["iter"] == 1


def test_warm_start_from_optimum(pm):
    """Section 6: warm start at the oracle's solution solves at the first check."""
    qp = qpgen.config_instance(1, 3)
    r = oracle.solve(qp)
    s = pm.Solver(qp, precision="fp64")
    s.warm_start(r.x, r.y)
    s.solve()
    x, y, info = s.result()
    s.close()
    assert info["status_name"] == "solved" and info["iter"] <= 25


def test_update_vectors_matches_fresh_setup(pm):
    """Section 6: new l, u (MPC initial state) through osqp_update_vectors
    give the oracle's solution of the updated problem."""
    rng = qpgen.rng_for(3, 500)
    plant = qpgen.mpc_plant(rng)
    qp0 = qpgen.mpc(rng, T=10, plant=plant)
    qp1 = qpgen.mpc(rng, T=10, plant=plant)   # same matrices, new x_init
    s = pm.Solver(qp0, precision="fp32")
    s.solve()
    s.update_vectors(l=qp1.l, u=qp1.u)
    s.solve()
    x, y, info = s.result()
    s.close()
    gc.compare(qp1, x, y, info, oracle.solve(qp1))


def test_subset_solve(pm):
    """osqp_batch_solve_subset_async: new l, u for two QPs of a resident
    batch (same plants, new initial states), re-solved as a subset, give the
    oracle's solutions of the updated problems; the other QPs' results stay
    bitwise as they were."""
    plants = [qpgen.mpc_plant(qpgen.rng_for(3, 600 + i)) for i in range(5)]
    qps = [qpgen.mpc(qpgen.rng_for(3, 700 + i), T=8, plant=plants[i]) for i in range(5)]
    new = {1: qpgen.mpc(qpgen.rng_for(3, 800), T=8, plant=plants[1]),
           3: qpgen.mpc(qpgen.rng_for(3, 801), T=8, plant=plants[3])}
    b = pm.Batch(qps, precision="fp32")
    b.solve()
    before = [b.get(i) for i in range(5)]
    for i, q in new.items():
        b.update_vectors(i, l=q.l, u=q.u)
    b.solve_subset(sorted(new))
    after = [b.get(i) for i in range(5)]
    b.close()
    for i in range(5):
        if i in new:
            gc.compare(new[i], *after[i], oracle.solve(new[i]))
        else:
            assert np.array_equal(before[i][0], after[i][0])
            assert np.array_equal(before[i][1], after[i][1])


def test_deterministic_and_alone_equals_mix(pm):
    """The same QP gives bitwise-identical results when solved twice, and
    alone or inside a batch of other QPs (one QP per workgroup, fixed
    reduction order)."""
    target = qpgen.config_instance(3, 7)
    others = [qpgen.config_instance(3, i) for i in range(20, 40)]
    xa, ya, ia = _solve_batch(pm, [target], precision="fp32")[0]
    xb, yb, ib = _solve_batch(pm, [target], precision="fp32")[0]
    mix = _solve_batch(pm, others[:10] + [target] + others[10:], precision="fp32")
    xm, ym, im = mix[10]
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert np.array_equal(xa, xm) and np.array_equal(ya, ym)
    assert ia["iter"] == im["iter"] and ia["status"] == im["status"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_polish_after_the_whole_grid_team(pm, precision):
    """A QP large enough for the whole-grid team (Jacobi PCG on every
    workgroup of a cooperative launch; the graph path refuses such a batch,
    which shows the team it runs on) is polished afterwards on one
    workgroup: the oracle's status and objective, and where both polishes
    are accepted the polished objectives agree to 1e-6."""
    qp = qpgen.config_instance(1, 0, n=350, m=3500)
    print(f"grid team + polish {precision}", flush=True)
    b = pm.Batch([qp], precision=precision, linsys="pcg", polish=1)
    with pytest.raises(pm.OSQPError) as e:
        b.solve_graph()
    assert e.value.code == 13
    b.solve()
    x, y, info = b.get(0)
    b.close()
    ref = oracle.solve(qp, polish=1)
    row = gc.compare(qp, x, y, info, ref)
    gc.assert_obj_parity([row], f"grid team + polish {precision}")
    print(f"  polish: device {info['polish_status']}, oracle {ref.polish_status}", flush=True)
    if info["polish_status"] == 1 and ref.polish_status == 1:
        assert row["obj_err"] <= 1e-6, row["obj_err"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lowrank_beyond_the_lds_stage(pm, precision):
    """The low-rank (Woodbury) path on a factor-model portfolio too large for
    the LDS stage (4000 assets: n = 4400, m = 4401), so every gather of its
    direct step comes from memory: the oracle's status and objective, one
    direct step per ADMM iteration, the oracle's iteration count in FP64."""
    qp = qpgen.portfolio(qpgen.rng_for(4, 4000), n=4000)
    ref = oracle.solve(qp)
    x, y, info = pm.solve(qp, precision=precision)
    assert info["linsys"] == 3
    row = gc.compare(qp, x, y, info, ref)
    gc.assert_obj_parity([row], f"{qp.name} {precision}")
    assert info["pcg_iter"] == info["iter"]
    if precision == "fp64":
        assert info["iter"] == ref.iter


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dense_path_at_its_limits(pm, precision):
    """The dense path at its size limits, on QPs the oracle factors cheaply
    (tridiagonal P, six dense rows of A, a box): n = 3000, the largest QP
    polished through the dense condensed system (47 diagonal blocks of 64),
    where the polished point is the oracle's; and n = 4096, the largest QP
    given the dense factor on request, where polishing is reported as not
    run.  Both take the oracle's status and objective with one exact step
    per ADMM iteration."""
    for n, polish_expected in ((3000, None), (4096, 0)):
        qp = qpgen.few_dense_rows(np.random.default_rng(11), n)
        print(f"dense limit n={n} {precision}", flush=True)
        ref = oracle.solve(qp, polish=1)
        x, y, info = pm.solve(qp, precision=precision, linsys="dense", polish=1)
        assert info["linsys"] == 2
        row = gc.compare(qp, x, y, info, ref)
        gc.assert_obj_parity([row], f"dense limit n={n} {precision}")
        assert info["pcg_iter"] == info["iter"]
        if polish_expected is None:
            assert info["polish_status"] == ref.polish_status == 1
            assert np.max(np.abs(x - ref.x)) <= 1e-8 * max(1.0, np.max(np.abs(ref.x)))
        else:
            assert info["polish_status"] == polish_expected


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_lasso_full_size_grid_team(pm, precision):
    """Workload 2 (Lasso, 10000 x 2000 at 5%): one QP on the whole grid."""
    qp = qpgen.config_instance(2, 0)
    print(f"lasso full {precision}", flush=True)
    x, y, info = pm.solve(qp, precision=precision)
    ref = oracle.solve(qp)
    row = gc.compare(qp, x, y, info, ref)
    print(f"lasso full {precision}: it={info['iter']} pcg={info['pcg_iter']} "
          f"obj_err={row['obj_err']:.2e}", flush=True)
    gc.assert_obj_parity([row], f"lasso full {precision}")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_polish_matches_brute_force(pm, precision):
    """Section 4 on tiny QPs: the device's FP64 polish (dense condensed
    Cholesky + iterative refinement) reproduces the enumerated optimum."""
    from tests.test_oracle_pins import _tiny_random
    qps = [_tiny_random(s) for s in range(40)]
    print(f"polish tiny x40 {precision}", flush=True)
    res = _solve_batch(pm, qps, precision=precision, polish=1)
    ok = 0
    for qp, (x, y, info) in zip(qps, res):
        x_bf, _, f_bf = qpcheck.brute_force(qp)
        assert info["status_name"] == "solved"
        if info["polish_status"] == 1:
            ok += 1
            assert np.allclose(x, x_bf, atol=1e-7), qp.name
            assert abs(info["obj_val"] - f_bf) <= 1e-8 * max(1.0, abs(f_bf)), qp.name
    print(f"polish accepted on {ok} of 40", flush=True)
    assert ok >= 30


def _polished_parity(pm, qps, label, precision):
    """Polish on both sides.  Where both polishes are accepted they started
    from the same active-set guess, so the polished points agree to 1e-6.
    Every instance is held to the objective bar (1e-3, else the
    eps-consistency verdict against the eps = 1e-8 optimum); polish is
    accepted on one side only for at most a tenth of the instances."""
    res = _solve_batch(pm, qps, precision=precision, polish=1)
    rows, mixed, both = [], 0, 0
    for qp, (x, y, info) in zip(qps, res):
        ref = oracle.solve(qp, polish=1)
        row = gc.compare(qp, x, y, info, ref)
        gp, op = info["polish_status"] == 1, ref.polish_status == 1
        if gp and op:
            both += 1
            assert row["obj_err"] <= 1e-6, (qp.name, row["obj_err"])
        elif gp != op:
            mixed += 1
        rows.append(row)
    errs = [r["obj_err"] for r in rows if "obj_err" in r]
    print(f"{label}: both polished {both}/{len(qps)}, one-sided {mixed}, "
          f"max obj err {max(errs):.2e}", flush=True)
    gc.assert_obj_parity(rows, label)
    assert mixed <= max(1, len(qps) // 10)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_random_qp_100_seeds_polished(pm, precision):
    """Workload 1 with polishing on both sides."""
    _polished_parity(pm, [qpgen.config_instance(1, i) for i in range(100)],
                     f"random_qp x100 polished {precision}", precision)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_portfolio_polished_parity(pm, precision):
    """Workload 4 generator with FP64 polish."""
    _polished_parity(pm, [qpgen.config_instance(4, i, n_range=(100, 800)) for i in range(12)],
                     f"portfolio x12 polished {precision}", precision)


LINSYS_CODE = {"pcg": 1, "dense": 2, "lowrank": 3, "band": 4}


@pytest.mark.parametrize("linsys", ["dense", "pcg", "lowrank", "band"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_linear_system_paths_agree(pm, linsys, precision):
    """The reduced-system solvers -- PCG preconditioned by the dense Cholesky
    factor of P + sigma I + A'RA or by its diagonal, the direct steps of its
    diagonal-plus-low-rank (Woodbury) form and of its block-tridiagonal
    factor after a reverse Cuthill-McKee ordering -- reach the oracle's
    status and objective on MPC and portfolio instances.  The low-rank form
    is taken where P is diagonal and A has at most n/2 multi-entry rows (the
    portfolios); the MPC instances, with more dynamics rows, fall back to the
    band factor (half-bandwidth 49 after the ordering) or, where that would
    not be smaller (T = 5), the dense one.  The portfolios have a dense row
    (1'x = 1), so the band setting gives them the low-rank form."""
    qps = [qpgen.config_instance(3, i) for i in range(8)] + \
          [qpgen.config_instance(4, i, n_range=(100, 400)) for i in range(4)]
    print(f"linsys={linsys} {precision}", flush=True)
    res = _solve_batch(pm, qps, precision=precision, linsys=linsys)
    rows = [gc.compare(q, *r, oracle.solve(q)) for q, r in zip(qps, res)]
    gc.summarize(rows, f"linsys={linsys} {precision}")
    gc.assert_obj_parity(rows, f"linsys={linsys} {precision}",
                         repolish=lambda q: pm.solve(q, precision=precision, linsys=linsys,
                                                     polish=1))
    its = [r[2]["pcg_iter"] / max(1, r[2]["iter"]) for r in res]
    print(f"  mean pcg per admm step {np.mean(its):.2f}", flush=True)
    paths = [r[2]["linsys"] for r in res]
    if linsys in ("lowrank", "band"):
        assert paths[8:] == [3] * 4, paths
        assert all(p in (2, 4) for p in paths[:8]) and 4 in paths[:8], paths
    else:
        assert paths == [LINSYS_CODE[linsys]] * len(qps), paths
    if precision == "fp64" and linsys != "pcg":
        # exact factors: the oracle's iteration counts
        for q, r in zip(qps, res):
            assert r[2]["iter"] == oracle.solve(q).iter, q.name


def test_auto_path_choice(pm):
    """Under the default (auto) choice the factor-model portfolios get the
    low-rank form, MPC QPs with T >= 10 the band factor, random QPs (P not
    diagonal, long rows) the dense factor."""
    qps = [qpgen.config_instance(4, i, n_range=(100, 600)) for i in range(3)] + \
          [qpgen.mpc(qpgen.rng_for(3, 40 + i), T=10 + 5 * i) for i in range(2)] + \
          [qpgen.config_instance(1, i) for i in range(2)]
    res = _solve_batch(pm, qps)
    assert [r[2]["linsys"] for r in res] == [3, 3, 3, 4, 4, 2, 2]


@pytest.mark.parametrize("linsys", ["dense", "band"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_factor_is_cholesky_of_reduced_matrix(pm, precision, linsys):
    """The MFMA-formed, MFMA-factored dense matrix and the band factor (block
    bidiagonal after the reverse Cuthill-McKee ordering, FP64): L L' equals
    Pbar + sigma I + Abar' R Abar recomputed in numpy from the scaled data
    (scaling from the oracle's independent Ruiz, same passes and readings)."""
    if linsys == "dense":
        qps = [qpgen.config_instance(1, 0), qpgen.config_instance(3, 1),
               qpgen.config_instance(4, 2, n_range=(100, 300))]
    else:
        qps = [qpgen.mpc(qpgen.rng_for(3, 70 + i), T=8 + 6 * i) for i in range(3)]
    b = pm.Batch(qps, precision=precision, linsys=linsys, max_iter=1, adaptive_rho=0)
    b.solve()
    for i, qp in enumerate(qps):
        assert b.get(i)[2]["linsys"] == LINSYS_CODE[linsys]
        L = b.factor(i)
        D, E, c = oracle.ruiz(qp, 10)
        Pb = c * (D[:, None] * qp.full_P().toarray() * D[None, :])
        Ab = E[:, None] * qp.A.toarray() * D[None, :]
        rho = np.where(qp.l == qp.u, 1e3 * 0.1, 0.1)
        K = Pb + 1e-6 * np.eye(qp.n) + Ab.T @ (rho[:, None] * Ab)
        err = np.max(np.abs(L @ L.T - K)) / np.max(np.abs(K))
        # the band factor is FP64 in both precisions, from the FP32 copies of
        # the scaled data in the FP32 path
        tol = 2e-5 if precision == "fp32" else 1e-12
        print(f"  {qp.name} {precision}: rel err of L L' {err:.2e}", flush=True)
        assert err <= tol, err
    b.close()
