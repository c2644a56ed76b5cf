"""Runs QPs through the host build of the library (its kernels executed on
the CPU by the SIMT stand-in, every device access address-sanitized) and
compares each result with the oracle.  Started by the CPU test in a process
of its own, with the sanitizer runtime preloaded:

    python tests/simt/runner.py [CASE ...]

Prints one line per check ("ok ..." or "FAIL ...") and exits non-zero if a
check fails; a sanitizer report aborts the process."""
from __future__ import annotations

import ctypes
import os
import sys
import time
import traceback

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import scipy.sparse as sp  # noqa: E402

import oracle  # noqa: E402
import paper_1711_08013_amd as pm  # noqa: E402
import qpgen  # noqa: E402
from qpgen import QP  # noqa: E402
from tests import gpu_common as gc  # noqa: E402


def load():
    """Bind the package's binding to the host build."""
    pm._lib = pm._configure(ctypes.CDLL(os.path.join(HERE, "_build", "libosqp_simt.so")))
    return pm._lib


def _same_as_oracle(qp, res, exact_iters, objective=True, **kw):
    """Status, eps test and objective as the GPU parity tests require (the
    objective within 1e-3 of the oracle's, else eps-consistent); on the
    exact-factor paths in FP64 also the oracle's iteration count."""
    x, y, info = res
    ref = oracle.solve(qp, **kw)
    ek = {k: kw[k] for k in ("eps_abs", "eps_rel") if k in kw}
    row = gc.compare(qp, x, y, info, ref, **ek)
    if objective and "obj_err" in row:
        gc.assert_obj_parity([row], qp.name)
    if exact_iters:
        assert info["iter"] == ref.iter, (qp.name, info["iter"], ref.iter)
    return info


def case_paths():
    """Dense factor, low-rank (Woodbury), band and Jacobi-PCG paths, both
    precisions; the exact factors take the oracle's iteration counts in FP64
    (the band and low-rank steps are FP64 in both precisions)."""
    qps = {"dense": qpgen.random_qp(20, qpgen.rng_for(9, 1)),
           "lowrank": qpgen.config_instance(4, 0, n_range=(100, 101)),
           "band": qpgen.mpc(qpgen.rng_for(3, 6), T=12),
           "pcg": qpgen.random_qp(20, qpgen.rng_for(9, 2))}
    code = {"pcg": 1, "dense": 2, "lowrank": 3, "band": 4}
    for path, qp in qps.items():
        for prec in ("fp64", "fp32"):
            res = pm.solve(qp, precision=prec, linsys=path)
            assert res[2]["linsys"] == code[path], (path, res[2]["linsys"])
            _same_as_oracle(qp, res, exact_iters=(prec == "fp64" and path != "pcg"))
            if path in ("band", "lowrank") or (path == "dense" and prec == "fp64"):
                assert res[2]["pcg_iter"] == res[2]["iter"], res[2]   # one direct step each
            yield f"{path} {prec} iter {res[2]['iter']}"


def case_mpc():
    qp = qpgen.mpc(qpgen.rng_for(3, 5), T=5)
    res = pm.solve(qp, precision="fp64")
    _same_as_oracle(qp, res, exact_iters=True)
    yield f"mpc T=5 fp64 iter {res[2]['iter']}"


def case_polish():
    """FP64 polishing, dense and low-rank condensed forms."""
    for qp in (qpgen.random_qp(15, qpgen.rng_for(9, 3)),
               qpgen.config_instance(4, 1, n_range=(100, 101))):
        for prec in ("fp64", "fp32"):
            res = pm.solve(qp, precision=prec, polish=1)
            ref = oracle.solve(qp, polish=1)
            row = gc.compare(qp, *res, ref)
            if res[2]["polish_status"] == 1 and ref.polish_status == 1:
                assert row["obj_err"] <= 1e-6, (qp.name, row["obj_err"])
            yield f"polish {qp.name} {prec} status {res[2]['polish_status']}"


def case_polish_batch():
    """Forty tiny QPs polished in one batch: a workgroup polishes several QPs
    in turn, QPs with multi-entry active rows next to QPs without (the
    count of those rows must not leak from one QP to the next); each
    accepted polish is the enumerated optimum."""
    from tests import qpcheck
    from tests.test_oracle_pins import _tiny_random
    qps = [_tiny_random(s) for s in range(40)]
    mixed = {bool(np.any(np.diff(q.A.indptr) > 1)) for q in qps}
    assert mixed == {True, False}, mixed
    for prec in ("fp32", "fp64"):
        b = pm.Batch(qps, precision=prec, polish=1)
        b.solve()
        ok = 0
        for i, qp in enumerate(qps):
            x, y, info = b.get(i)
            assert info["status_name"] == "solved", (qp.name, info["status_name"])
            if info["polish_status"] == 1:
                ok += 1
                x_bf, _, f_bf = qpcheck.brute_force(qp)
                assert np.allclose(x, x_bf, atol=1e-7), qp.name
                assert abs(info["obj_val"] - f_bf) <= 1e-8 * max(1.0, abs(f_bf)), qp.name
        b.close()
        assert ok >= 30, ok
        yield f"polish batch x40 {prec} accepted {ok}"


def case_shapes():
    """Every launch shape osqp_batch_set_shape accepts for the solve
    (workgroups of 256 and 512 threads, lane divisors 8..64) on a small
    mixed batch: each matches the oracle and repeats bitwise; the tuner
    entry point is switched off (OSQP_ERR_UNSUPPORTED)."""
    qps = ([qpgen.random_qp(6, qpgen.rng_for(9, 10 + i)) for i in range(2)] +
           [qpgen.config_instance(4, 2, n_range=(100, 101))])
    b = pm.Batch(qps, precision="fp32")
    try:
        b.autotune(reps=1)
        raise AssertionError("the tuner entry point should be switched off")
    except pm.OSQPError as e:
        assert e.code == 13, e.code
    shapes = 0
    for block in (256, 512):
        for div in (8, 16, 32, 64):
            b.set_shape(block, div)
            b.reset()
            b.solve()
            r1 = [b.get(i) for i in range(len(qps))]
            b.reset()
            b.solve()
            r2 = [b.get(i) for i in range(len(qps))]
            for (xa, ya, _), (xb, yb, _) in zip(r1, r2):
                assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
            for qp, r in zip(qps, r1):
                _same_as_oracle(qp, r, exact_iters=False)
            shapes += 1
    b.close()
    yield f"set_shape over {shapes} shapes, each matching the oracle"


def case_graph():
    """Replays of the solve graph against the eager solve, bitwise, with
    eager work between the replays; after a new launch shape the graph is
    rebuilt and again matches."""
    qps = ([qpgen.random_qp(10, qpgen.rng_for(9, 20 + i)) for i in range(2)] +
           [qpgen.config_instance(4, 3, n_range=(100, 101)), qpgen.mpc(qpgen.rng_for(3, 6), T=5)])

    def same(ra, rb):
        for (xa, ya, ia), (xb, yb, ib) in zip(ra, rb):
            assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
            assert ia["iter"] == ib["iter"] and ia["polish_status"] == ib["polish_status"]

    b = pm.Batch(qps, precision="fp32", polish=1)
    b.solve()
    eager = [b.get(i) for i in range(len(qps))]
    for _ in range(2):
        b.reset()
        b.solve_subset([1, 3])
        b.reset()
        b.solve_graph()
        same(eager, [b.get(i) for i in range(len(qps))])
    b.set_shape(512, 16)
    b.reset()
    b.solve()
    eager2 = [b.get(i) for i in range(len(qps))]
    b.reset()
    b.solve_graph()
    same(eager2, [b.get(i) for i in range(len(qps))])
    b.close()
    for qp, r in zip(qps, eager):
        _same_as_oracle(qp, r, exact_iters=False, polish=1)
    yield "graph replays bitwise as eager, rebuilt after a shape change"


def case_grid():
    """QPs large enough for the whole-grid team (cooperative launch, grid
    barriers, two-level reductions): one whose vectors fit the LDS stage
    (n = 400, m = 4000; FP64, 50 ADMM iterations) and one too large for any
    staging, every gather from memory (n = 1000, m = 16000; FP32, 25
    iterations).  The oracle's status and an objective near its iterate's
    (the Jacobi inner solves are inexact); the solve graph is refused."""
    cases = [(qpgen.config_instance(1, 0, n=400, m=4000), "fp64", 50),
             (qpgen.random_qp(1000, qpgen.rng_for(9, 77), m=16000, density=0.01), "fp32", 25)]
    for qp, prec, iters in cases:
        b = pm.Batch([qp], precision=prec, linsys="pcg", max_iter=iters)
        try:
            b.solve_graph()
            raise AssertionError("graph accepted for a whole-grid QP")
        except pm.OSQPError as e:
            assert e.code == 13, e.code
        b.solve()
        x, y, info = b.get(0)
        b.close()
        ref = oracle.solve(qp, max_iter=iters)
        assert info["status_name"] == ref.status == "max_iter_reached", (info["status_name"], ref.status)
        assert np.isfinite(x).all() and np.isfinite(y).all()
        err = abs(info["obj_val"] - ref.obj_val) / max(1.0, abs(ref.obj_val))
        assert err <= 1e-2, err
        yield f"grid team {qp.name} {prec}: obj {info['obj_val']:.6f} (oracle {ref.obj_val:.6f})"


def case_server():
    """The continuous-batching server: fresh QPs, and a repeated structure
    (same key, new expected returns) re-solved warm in its resident pool."""
    rng = qpgen.rng_for(4, 901)
    F, Dd, mu = qpgen.portfolio_model(rng, 100)
    reqs = [(qpgen.random_qp(8, qpgen.rng_for(9, 30 + i)), 0) for i in range(3)]
    # a fresh QP above the server's size threshold (a launch of its own)
    reqs.append((qpgen.portfolio(qpgen.rng_for(4, 902), n=1500), 0))
    for _ in range(3):
        mu = 0.8 * mu + 0.2 * rng.standard_normal(mu.size)
        reqs.append((qpgen.portfolio(rng, model=(F, Dd, mu)), 7))
    with pm.Server(hbm_budget_bytes=1 << 30, max_slots=16) as sv:
        tickets = [sv.submit(qp, key=k) for qp, k in reqs]
        outs = [sv.wait(t) for t in tickets]
        stats = sv.stats()
        # a ticket is collected once (OSQP_ERR_INDEX from the C entry point)
        rc = pm.lib().osqp_server_wait(sv._h, ctypes.c_uint64(tickets[0]), None, None, None, None)
        assert rc == 11, rc
    assert stats["completed"] == len(reqs), stats
    # every request: the oracle's status, the eps test and the objective bar
    # (warm re-solves of the pool may stop at another eps-solution; they are
    # then held to the eps-consistency verdict against the eps = 1e-8 optimum)
    rows = []
    for (qp, key), (x, y, info, lat) in zip(reqs, outs):
        rows.append(gc.compare(qp, x, y, info, oracle.solve(qp)))
    gc.assert_obj_parity(rows, "server")
    yield f"server: {stats['completed']} requests in {stats['batches']} launches"
    _, st = gc.server_pool_kept_while_chosen(pm)
    yield f"server: a pool chosen for a repeat is kept under budget pressure ({st['batches']} launches)"


def case_server_estimate():
    """The server admits a request by an estimate of its device memory, which
    must bound what the request's batch allocates: a counting allocator
    installed with osqp_set_allocator records the peak of live bytes while
    each request is solved alone, for the reduced-system paths the estimate
    distinguishes (dense, low-rank with low-rank polishing, band below and
    above n = 2500, Jacobi)."""
    libc = ctypes.CDLL(None)
    libc.malloc.restype = ctypes.c_void_p
    libc.malloc.argtypes = [ctypes.c_size_t]
    libc.free.argtypes = [ctypes.c_void_p]
    live, peak = {}, [0]

    def alloc(nbytes):
        p = libc.malloc(nbytes)
        live[p] = nbytes
        peak[0] = max(peak[0], sum(live.values()))
        return p

    def free(p):
        del live[p]
        libc.free(p)

    cases = [(qpgen.random_qp(60, qpgen.rng_for(5, 1)), {}, 2),
             (qpgen.portfolio(qpgen.rng_for(4, 5), n=200), {"polish": 1}, 3),
             (qpgen.mpc(qpgen.rng_for(3, 6), T=12), {}, 4),
             (qpgen.banded(np.random.default_rng(5), 3000, 16), {}, 4),
             (qpgen.random_qp(60, qpgen.rng_for(5, 2)), {"linsys": "pcg"}, 1)]
    for qp, settings, path in cases:
        peak[0] = 0
        pm.set_allocator(alloc, free)
        try:
            with pm.Server(hbm_budget_bytes=64 << 30, max_slots=4, **settings) as sv:
                x, y, info, _ = sv.wait(sv.submit(qp))
                est = sv.stats()["peak_bytes"]
        finally:
            pm.set_allocator()
        assert info["linsys"] == path, (qp.name, info["linsys"])
        assert not live, "an allocation was not returned"
        assert 0 < peak[0] <= est, (qp.name, peak[0], est)
        yield f"server estimate {qp.name}: {peak[0] / 1e6:.2f} MB used <= {est / 1e6:.2f} MB"
    # an FP64 server with polishing: fresh QPs and repeats of one key, each
    # result the polished oracle's status and objective
    plant = qpgen.mpc_plant(qpgen.rng_for(3, 70))
    reqs = [(qpgen.random_qp(15, qpgen.rng_for(9, 71)), 0),
            (qpgen.portfolio(qpgen.rng_for(4, 72), n=150), 0),
            (qpgen.mpc(qpgen.rng_for(3, 73), T=6, plant=plant), 5),
            (qpgen.mpc(qpgen.rng_for(3, 74), T=6, plant=plant), 5)]
    with pm.Server(hbm_budget_bytes=1 << 30, max_slots=8, precision="fp64", polish=1) as sv:
        outs = [sv.wait(t) for t in [sv.submit(qp, key=k) for qp, k in reqs]]
    rows = [gc.compare(qp, x, y, info, oracle.solve(qp, polish=1))
            for (qp, _), (x, y, info, _) in zip(reqs, outs)]
    gc.assert_obj_parity(rows, "server fp64 polish")
    yield f"server fp64 with polishing: {len(reqs)} requests"


def case_edges():
    """Scalar QP, no constraints, A = I, LP, empty and free rows."""
    e = dict(eps_abs=1e-6, eps_rel=1e-6, max_iter=50000)
    scalar = QP(sp.csr_matrix([[2.0]]), np.array([-4.0]), sp.csr_matrix([[1.0]]),
                np.array([-1.0]), np.array([1.0]), name="scalar")
    rng = np.random.default_rng(11)
    M = rng.standard_normal((6, 6))
    m0 = QP(sp.csr_matrix(np.triu(M @ M.T + np.eye(6))), rng.standard_normal(6),
            sp.csr_matrix((0, 6)), np.zeros(0), np.zeros(0), name="m=0")
    box = qpgen.box_qp(rng.uniform(0.1, 2.0, 9), rng.standard_normal(9), -np.ones(9), np.ones(9))
    q = rng.standard_normal(8)
    lp = QP(sp.csr_matrix((8, 8)), q, sp.identity(8, format="csr"), -np.ones(8), np.ones(8),
            name="box LP")
    base = qpgen.random_qp(10, qpgen.rng_for(9, 4))
    A = sp.vstack([base.A, sp.csr_matrix((2, base.n)),
                   sp.csr_matrix(rng.standard_normal((2, base.n)))], format="csr")
    rows = QP(base.P, base.q, A, np.concatenate([base.l, [-1.0, 0.0], [-np.inf] * 2]),
              np.concatenate([base.u, [1.0, 0.0], [np.inf] * 2]), name="empty+free rows")
    for qp in (scalar, m0, box, lp, rows):
        res = pm.solve(qp, precision="fp64", **e)
        if qp.m == 0:
            assert res[2]["status_name"] == "solved"
            xs = -np.linalg.solve(qp.full_P().toarray(), qp.q)
            assert np.allclose(res[0], xs, atol=1e-5)
        else:
            _same_as_oracle(qp, res, exact_iters=False, **e)
        yield f"edge {qp.name}"
    # all of them in one batch with a regular QP: bitwise as alone
    qps = [scalar, m0, box, lp, rows, base]
    b = pm.Batch(qps, precision="fp32")
    b.solve()
    mixed = [b.get(i) for i in range(len(qps))]
    b.close()
    for qp, (x, y, _) in zip(qps, mixed):
        xa, ya, _ = pm.solve(qp, precision="fp32")
        assert np.array_equal(x, xa) and np.array_equal(y, ya), qp.name
    yield "edge batch bitwise as alone"


def case_certificates():
    A = sp.csr_matrix(np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
    pinf = QP(sp.csr_matrix(np.eye(2)), np.zeros(2), A, np.array([1.0, -np.inf, -1.0]),
              np.array([np.inf, 0.0, 1.0]), name="primal infeasible")
    dinf = qpgen.box_qp(np.zeros(5), -np.ones(5), np.zeros(5), np.inf * np.ones(5))
    for prec in ("fp64", "fp32"):
        assert pm.solve(pinf, precision=prec)[2]["status_name"] == "primal_infeasible"
        assert pm.solve(dinf, precision=prec)[2]["status_name"] == "dual_infeasible"
        yield f"certificates {prec}"


def case_appendix():
    """Equality QP, Huber fitting and SVM at small sizes."""
    for qp in (qpgen.eq_qp(12, qpgen.rng_for(9, 5)),
               qpgen.huber(qpgen.rng_for(7, 1), 2, m_data=24),
               qpgen.svm(qpgen.rng_for(7, 2), 2, m_data=24)):
        for prec in ("fp64", "fp32"):
            res = pm.solve(qp, precision=prec)
            _same_as_oracle(qp, res, exact_iters=False)
            yield f"{qp.name} {prec} linsys {res[2]['linsys']}"


def case_updates():
    """Vector and matrix updates with warm start (Section 6)."""
    qp = qpgen.random_qp(12, qpgen.rng_for(9, 6))
    s = pm.Solver(qp, precision="fp64")
    s.solve()
    q2 = qp.q + 0.1
    s.update_vectors(q=q2)
    s.solve()
    qpv = QP(qp.P, q2, qp.A, qp.l, qp.u, name="q updated")
    _same_as_oracle(qpv, s.result(), exact_iters=False)
    A2 = qp.A.copy()
    A2.data = A2.data * 1.1
    s.update_matrices(A=A2)
    s.solve()
    x, y, info = s.result()
    qpm = QP(qp.P, q2, A2, qp.l, qp.u, name="A updated")
    row = gc.compare(qpm, x, y, info, oracle.solve(qpm))
    assert row.get("obj_err", 0.0) <= gc.OBJ_TOL
    s.close()
    yield "updates"


def case_allocator():
    """osqp_set_allocator: every device allocation of a handle goes through
    the installed pair and is returned through it at cleanup; the results
    equal those with hipMalloc bitwise; only-one-of-the-pair is refused."""
    libc = ctypes.CDLL(None)
    libc.malloc.restype = ctypes.c_void_p
    libc.malloc.argtypes = [ctypes.c_size_t]
    libc.free.argtypes = [ctypes.c_void_p]
    live, calls = {}, [0, 0]

    def alloc(nbytes):
        p = libc.malloc(nbytes)
        live[p] = nbytes
        calls[0] += 1
        return p

    def free(p):
        assert p in live, "freed an address the allocator did not hand out"
        del live[p]
        calls[1] += 1
        libc.free(p)

    qps = [qpgen.random_qp(12, qpgen.rng_for(9, 60)), qpgen.mpc(qpgen.rng_for(3, 61), T=12)]
    ref = pm.Batch(qps, precision="fp32", polish=1)
    ref.solve()
    r0 = [ref.get(i) for i in range(len(qps))]
    ref.close()
    rc = pm.lib().osqp_set_allocator(pm._ALLOC_FN(lambda n, c: 0), pm._FREE_FN(), None)
    assert rc == 6, rc
    pm.set_allocator(alloc, free)
    try:
        b = pm.Batch(qps, precision="fp32", polish=1)
        b.solve()
        r1 = [b.get(i) for i in range(len(qps))]
    finally:
        pm.set_allocator()
    # the batch keeps the pair it was created with: closed after hipMalloc
    # is back, it still returns its memory through that pair
    import gc as _gc
    _gc.collect()
    b.close()
    assert calls[0] >= 4 and calls[0] == calls[1] and not live, (calls, live)
    for (xa, ya, _), (xb, yb, _) in zip(r0, r1):
        assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    yield f"allocator: {calls[0]} allocations through the hook, all returned"


CASES = {"paths": case_paths, "mpc": case_mpc, "polish": case_polish,
         "polish_batch": case_polish_batch, "server_estimate": case_server_estimate, "shapes": case_shapes,
         "graph": case_graph, "grid": case_grid,
         "server": case_server,
         "edges": case_edges, "certificates": case_certificates, "appendix": case_appendix,
         "updates": case_updates, "allocator": case_allocator}


def main(names):
    load()
    failed = 0
    for name in names or list(CASES):
        t0 = time.time()
        try:
            for msg in CASES[name]():
                print(f"ok {name}: {msg} ({time.time() - t0:.1f} s)", flush=True)
        except Exception:
            failed += 1
            print(f"FAIL {name}:\n{traceback.format_exc()}", flush=True)
    return 1 if failed else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
