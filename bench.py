#!/usr/bin/env python3
"""Benchmark of the batched FP32-mixed ADMM QP path on one MI355X.

A step is one pass of the whole hot path over one batch with the problem data
already resident in HBM: device-side Ruiz equilibration, rho vector and
preconditioner, the ADMM iterations with their reduced-system solves, FP64
termination / infeasibility checks and rho adaptation, unscaling (and
polishing when enabled), then the results copied to the host.

Prints one JSON line.  Beside the timed batch it reports, for every QP of the
batch, the error against the FP64 CPU oracle (which also gives the CPU
baseline: the oracle on a pool of host threads), the FP64 plain
single-instance GPU path, and optional legs (high accuracy, parametric
re-solves, a serving stream).  Only --gpus 1 is supported: the library drives
a single GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import qpgen  # noqa: E402

METRIC = "solved QPs/s + p99 latency at eps 1e-3, FP32 batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0
CHECK_EVERY = 25

WORKLOADS = {
    # name: (cfg, count, description, extra settings)
    "portfolio": (4, 1024, "batched factor-model portfolio, 1024 QPs, n in [100,2000], "
                           "k=n/10, F 50% dense, FP32 with FP64 polish", {"polish": 1}),
    "mpc": (3, 4096, "batched linear MPC, 4096 QPs, nx=20, nu=10, T in [5,20], FP32", {}),
    "lasso": (2, 1, "Lasso 10000 x 2000 at 5% as one QP (n = m = 14000) on the whole grid, "
                    "FP32 PCG with FP64 residuals", {}),
}
# the kernel whose launch time the roofline divides by
KERNEL = {"portfolio": "solve_wg_kernel<float>", "mpc": "solve_wg_kernel<float>",
          "lasso": "solve_grid_kernel<float>"}
# launch shape (workgroup size : lane divisor) applied before the timed
# steps: the fastest of the shapes timed earlier on each workload (the same
# workgroup size the setup picks, so the grid stays the setup's)
DEFAULT_SHAPES = {"portfolio": "512:32", "mpc": "256:32"}

# the serving configuration: Poisson arrivals, one third each of random QPs
# (n log-uniform, m = 10 n), MPC requests (64 plants) and portfolio requests
# (16 models); the first second of arrivals is discarded as warm-up
SERVING_FULL = {"requests": 20000, "rate": 2000.0, "n_max": 5000, "warmup_s": 1.0}


def build_workload(name: str, count: int | None):
    cfg, n_default, desc, extra = WORKLOADS[name]
    count = n_default if count is None else count
    qps = [qpgen.config_instance(cfg, i) for i in range(count)]
    return qps, desc, extra


def _sizes(qp):
    """n, m, a = nnz(A), p = nnz(P full), a_m entries of A's multi-entry rows,
    R = number of those rows."""
    n, m = qp.n, qp.m
    a = int(qp.A.nnz)
    p = int(2 * qp.P.nnz - int((qp.P.diagonal() != 0).sum()))
    rl = np.diff(qp.A.indptr)
    return n, m, a, p, int(rl[rl >= 2].sum()), int((rl >= 2).sum())


def s8d_bytes(qp, info, check_every: int = CHECK_EVERY) -> float:
    """Algorithmic bytes of one QP's solve: what the method must read, each
    matrix once per application, FP32 values with int32 indices (8 B per
    entry), FP64 values in the checks (12 B per entry).  Per PCG iteration
    (two passes: A, then A' and P) 16a + 8p + 4(12n + 4m); per ADMM
    iteration (k_pcg + 1) PCG iterations' worth (the right-hand side is one
    more pass) plus 4(5n + 12m) for the vector update; per termination check
    12(2a + p) + 8(6n + 6m).  k_pcg is the QP's mean inner steps per ADMM
    step (an exact reduced-system solve counts as one).  No factor is
    counted: the reduced matrix the method avoids forming is not
    algorithmic traffic."""
    n, m, a, p, _, _ = _sizes(qp)
    it, pcg = int(info["iter"]), int(info["pcg_iter"])
    pcg_b = 16 * a + 8 * p + 4 * (12 * n + 4 * m)
    checks = -(-it // check_every)
    return float((pcg + it) * pcg_b + it * 4 * (5 * n + 12 * m) +
                 checks * (12 * (2 * a + p) + 8 * (6 * n + 6 * m)))


def algorithmic_bytes(qps, infos, check_every: int = CHECK_EVERY) -> float:
    return float(sum(s8d_bytes(q, i, check_every) for q, i in zip(qps, infos)))


def path_bytes(qps, infos, value_bytes=4, check_every=CHECK_EVERY):
    """Bytes this implementation's passes move, summed over the batch (for
    comparison with the algorithmic bytes; includes what the method does not
    need, such as the dense factor's n^2 applies).  Per QP with e = 4 + vb
    (index + working-precision value):
      ADMM iteration : start pass A', P -> e (a + p) + 8 (6n + m);
                       update pass A    -> e a + 8 (3n + 9m)
      low-rank path  : one direct apply per iteration (counted in pcg_iter)
                       -> e (a_m + a) + 8 (R^2 + 4n + 2m); no PCG products
      band path      : one direct step per iteration (counted in pcg_iter),
                       each sweep over the nonzero triangles of the FP64
                       tiles -> 16 nb n + 8 (3n); no PCG products
      dense path     : PCG iterations e (2a + p) + 4 (2n + m) + vb (5n + 2m) + 16n,
                       applies (ADMM iterations + inner iterations beyond the
                       first) vb n^2 + 2 vb n; in FP64 (vb = 8) the factor
                       gives the direct step: one apply per iteration and
                       no PCG products
      Jacobi path    : PCG iterations as above, no applies
      check (FP64, every 25 iterations): 12 (2a + p) + 8 (6n + 6m)
      factorisation (1 + rho updates): low-rank 8 (2 R n + R^2) + e a_m;
                                       band 16 nb n + e (a + p);
                                       dense 3 vb n^2
    The band block size nb is bounded by 64 (the value used here; the
    ordering usually gives 56 on the MPC workload)."""
    vb = value_bytes
    e = 4 + vb
    total = 0.0
    for qp, info in zip(qps, infos):
        n, m, a, p, am, R = _sizes(qp)
        it, pcg = info["iter"], info["pcg_iter"]
        admm = it * (e * (a + p) + 8 * (6 * n + m) + e * a + 8 * (3 * n + 9 * m))
        pcg_b = e * (2 * a + p) + 4 * (2 * n + m) + vb * (5 * n + 2 * m) + 16 * n
        path = info.get("linsys", 1)
        if path == 3:
            work = pcg * (e * (am + a) + 8 * (R * R + 4 * n + 2 * m))
            fact_b = 8 * (2 * R * n + R * R) + e * am
        elif path == 4:
            nb = 64
            work = pcg * (16 * nb * n + 8 * 3 * n)
            fact_b = 16 * nb * n + e * (a + p)
        elif path == 2 and vb == 8:
            work = pcg * (vb * n * n + 2 * vb * n)
            fact_b = 3 * vb * n * n
        elif path == 2:
            work = pcg * pcg_b + (it + max(0, pcg - it)) * (vb * n * n + 2 * vb * n)
            fact_b = 3 * vb * n * n
        else:
            work = pcg * pcg_b
            fact_b = 0
        checks = -(-it // check_every)
        chk = checks * (12 * (2 * a + p) + 8 * (6 * n + 6 * m))
        total += admm + work + chk + (1 + info["rho_updates"]) * fact_b
    return float(total)


# the headers that hold device code (the kernels and what they include);
# api.hip and server.h are host code
KERNEL_SOURCES = ("dense.h", "kernels.h", "polish.h", "qp_layout.h", "solver_device.h", "team.h")


def kernel_source_sha256() -> str:
    """Hash of the device-code sources, to tie a stored counter measurement
    to the kernels it was taken on (the launch shape is recorded beside it)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1711_08013_amd", "csrc")
    files = [os.path.join(csrc, f) for f in KERNEL_SOURCES]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(workload: str, shape):
    """HBM bytes per solve launch from the committed counter summary of this
    workload, if it was taken on the current kernel sources and at the launch
    shape (block size, lane divisor) the timed steps ran with; else None."""
    path = os.path.join(ROOT, "profiles", f"solve_wg_kernel_{workload}1024_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and line.split("=")[0].strip() in ("traffic_bytes_per_launch",
                                                              "kernel_source_sha256",
                                                              "launch_shape"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    if shape is None or vals.get("launch_shape") != f"{shape[0]}:{shape[1]}":
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# host, oracle and error report
# ---------------------------------------------------------------------------
def host_threads(cap: int = 16) -> int:
    """Host threads for the oracle pool: the CPUs this process may run on,
    at most `cap` (on a shared multi-GPU host, about one GPU's share of its
    cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def oracle_pool(qps, extra: dict, threads: int):
    """The FP64 CPU oracle as it stands on every QP, `threads` QPs at a time
    (one whole QP per task; the library call releases the interpreter lock).
    Returns the results and the wall time."""
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    pol = int(extra.get("polish", 0))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        refs = list(ex.map(lambda q: oracle.solve(q, polish=pol), qps))
    return refs, time.perf_counter() - t0


def p_positive_definite(qp) -> bool:
    """Whether P is known positive definite: diagonal with a positive
    diagonal, or (small n) by its smallest eigenvalue."""
    P = qp.P
    if P.nnz == int((P.diagonal() != 0).sum()):
        return bool(np.all(P.diagonal() > 0))
    if qp.n <= 300:
        return bool(np.linalg.eigvalsh(qp.full_P().toarray()).min() > 0)
    return False


def error_report(qps, results, refs, eps_abs=1e-3, eps_rel=1e-3):
    """Error of every GPU result against the oracle: status match; for QPs
    both sides solve, |f - f_or| / max(1, |f_or|), the eps-scaled FP64
    residuals recomputed on the host from the returned x, y (z = Pi(Ax)),
    and, where P is positive definite, ||x - x_or||_inf / max(1, ||x_or||_inf)."""
    from tests import qpcheck
    match = both = over = 0
    obj, rp_max, rd_max, xerr = 0.0, 0.0, 0.0, None
    for qp, (x, y, info), ref in zip(qps, results, refs):
        if info["status_name"] != ref.status:
            continue
        match += 1
        if ref.status != "solved":
            continue
        both += 1
        e = abs(info["obj_val"] - ref.obj_val) / max(1.0, abs(ref.obj_val))
        obj = max(obj, e)
        over += e > 1e-3
        rp, rd = qpcheck.eps_scaled_residuals(qp, x, y, eps_abs, eps_rel)
        rp_max, rd_max = max(rp_max, rp), max(rd_max, rd)
        if p_positive_definite(qp):
            d = float(np.max(np.abs(x - ref.x)) / max(1.0, np.max(np.abs(ref.x))))
            xerr = d if xerr is None else max(xerr, d)
    return {"qps": len(qps), "status_match": match, "both_solved": both,
            "max_rel_obj_err": obj, "obj_err_above_1e-3": over,
            "max_eps_scaled_prim": rp_max, "max_eps_scaled_dual": rd_max,
            "max_rel_x_err_p_definite": xerr}


def fp64_plain(pm, qps, budget_s: float, extra: dict):
    """The FP64 plain single-instance GPU path: same kernels in double, batch
    of one, QPs solved one after another on one stream."""
    times, solved = [], 0
    t_all = time.perf_counter()
    for qp in qps:
        s = pm.Solver(qp, precision="fp64", **extra)
        t0 = time.perf_counter()
        s.solve()
        times.append(time.perf_counter() - t0)
        solved += s.result()[2]["status_name"] == "solved"
        s.close()
        if time.perf_counter() - t_all >= budget_s:
            break
    return {"qps": solved / sum(times), "count": len(times),
            "p50_latency_ms": float(np.percentile(times, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(times, 99) * 1e3)}


def high_accuracy_leg(pm, qps, extra, shape):
    """The same batch at the paper's high-accuracy setting, eps = 1e-5."""
    hb = pm.Batch(qps, precision="fp32", eps_abs=1e-5, eps_rel=1e-5, max_iter=20000, **extra)
    try:
        if shape:
            hb.set_shape(*shape)
        hb.reset()
        t0 = time.perf_counter()
        hb.solve()
        hs = time.perf_counter() - t0
        hinf = [hb.get(i)[2] for i in range(len(qps))]
    finally:
        hb.close()
    hsolved = sum(1 for i in hinf if i["status_name"] == "solved")
    return {"eps": 1e-5, "solved": hsolved, "qps_per_s": round(hsolved / hs, 2),
            "batch_ms": round(hs * 1e3, 3),
            "mean_iter": round(float(np.mean([i["iter"] for i in hinf])), 1)}


def parametric_leg(pm):
    """Parametric re-solves (Section 6) on one QP each: a Lasso path of twelve
    lambda values (q updated, iterate kept) against cold solves, and an MPC
    closed loop of twenty steps (initial-state bounds updated); iterations and
    device time per re-solve."""
    out = {}
    base = qpgen.lasso(qpgen.rng_for(2, 11), 200, 2000, density=0.05, lam_frac=1.0)
    nf = 200
    fracs = np.geomspace(0.9, 0.05, 12)
    warm = pm.Solver(base, precision="fp32")
    warm.solve()
    it_w = it_c = 0
    ms_w = ms_c = 0.0
    for f in fracs:
        q = base.q.copy()
        q[-nf:] = f * base.lam
        warm.update_vectors(q=q)
        warm.solve()
        it_w += warm.result()[2]["iter"]
        ms_w += warm.last_kernel_ms()
        cold = pm.Solver(qpgen.QP(base.P, q, base.A, base.l, base.u), precision="fp32")
        cold.solve()
        it_c += cold.result()[2]["iter"]
        ms_c += cold.last_kernel_ms()
        cold.close()
    warm.close()
    out["lasso_path"] = {"problem": "Lasso 2000 x 200 at 5%, 12 lambda values in [0.05, 0.9] lambda_max",
                         "iters_warm": it_w, "iters_cold": it_c,
                         "kernel_ms_warm": round(ms_w, 3), "kernel_ms_cold": round(ms_c, 3)}
    rng = qpgen.rng_for(3, 901)
    plant = qpgen.mpc_plant(rng)
    Ad, B = plant[0], plant[1]
    nx, nu, T = 20, 10, 10
    x = rng.uniform(-1.0, 1.0, nx)
    s = pm.Solver(qpgen.mpc(rng, T=T, plant=plant, x_init=x), precision="fp32")
    its, ms = [], []
    for _ in range(20):
        s.solve()
        xs, _, info = s.result()
        its.append(info["iter"])
        ms.append(s.last_kernel_ms())
        x = Ad @ x + B @ xs[nx * (T + 1): nx * (T + 1) + nu]
        nq = qpgen.mpc(rng, T=T, plant=plant, x_init=x)
        s.update_vectors(l=nq.l, u=nq.u)
    s.close()
    out["mpc_closed_loop"] = {"problem": "MPC nx=20, nu=10, T=10, 20 steps",
                              "iters_mean": float(np.mean(its)),
                              "kernel_ms_p50": round(float(np.percentile(ms, 50)), 3),
                              "kernel_ms_p99": round(float(np.percentile(ms, 99)), 3)}
    return out


# ---------------------------------------------------------------------------
# serving stream
# ---------------------------------------------------------------------------
def serving_requests(n_req: int, rate: float, n_max: int, random_pool: int, seed_index: int = 0):
    """The serving workload's requests as (arrival time, QP, structure key).
    MPC and portfolio requests come from the generators as they are (repeats
    of a plant or model share its key).  Random QPs are fresh requests (key
    0: set up from scratch each time); their data is drawn from a pool of
    `random_pool` instances with n log-uniform in [20, n_max] (building a
    QP with n in the thousands takes the host seconds), each request taking
    the pool entry its own seeded draw names."""
    trace = qpgen.serving_trace(n_req, rate, seed_index=seed_index, n_range=(20, n_max))
    pool = [qpgen.serving_request({"kind": "random", "key": None, "index": 100000 + j}, {},
                                  n_range=(20, n_max)) for j in range(random_pool)]
    state, reqs = {}, []
    for r in trace:
        if r["kind"] == "random":
            j = int(qpgen.rng_for(5, r["index"]).integers(0, random_pool))
            reqs.append((r["t"], pool[j], 0))
        else:
            key = (1000 if r["key"][0] == "mpc" else 2000) + int(r["key"][1])
            reqs.append((r["t"], qpgen.serving_request(r, state, n_range=(20, n_max)), key))
    return reqs


def latency_stats(arrivals, latencies, warmup_s: float):
    """p50 / p99 (exact order statistics) of the requests that arrived after
    the warm-up window."""
    lat = np.array([l for t, l in zip(arrivals, latencies) if t >= warmup_s])
    if lat.size == 0:
        return None
    q = np.sort(lat)

    def order_stat(p):
        return float(q[min(q.size - 1, max(0, math.ceil(p * q.size) - 1))])

    return {"counted": int(lat.size), "p50_ms": round(order_stat(0.50) * 1e3, 3),
            "p99_ms": round(order_stat(0.99) * 1e3, 3)}


def run_stream(pm, reqs, warmup_s: float):
    """Submit the requests at their arrival times to a fresh server, wait for
    all; latency is the server's submit-to-completion time."""
    sv = pm.Server(hbm_budget_bytes=64 << 30, max_slots=1024, precision="fp32")
    start = time.perf_counter()
    tickets = []
    for t_arr, qp, key in reqs:
        delay = start + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(sv.submit(qp, key=key))
    outs = [sv.wait(t) for t in tickets]
    wall = time.perf_counter() - start
    stats = sv.stats()
    sv.close()
    arrivals = [r[0] for r in reqs]
    lats = [o[3] for o in outs]
    counted = [(t, o) for t, o in zip(arrivals, outs) if t >= warmup_s]
    solved = sum(1 for _, o in counted if o[2]["status_name"] == "solved")
    span = max(1e-9, wall - warmup_s)
    return {"requests": len(reqs), "wall_s": round(wall, 3),
            "arrival_span_s": round(arrivals[-1], 3),
            "throughput_qps": round(solved / span, 1), "solved_after_warmup": solved,
            "latency": latency_stats(arrivals, lats, warmup_s),
            "drain_s": round(wall - arrivals[-1], 3),
            "micro_batches": stats["batches"], "peak_inflight": stats["peak_inflight"]}


def sustainable(res: dict, rate: float, drain_s: float = 0.5) -> bool:
    """A rate is sustained when the server keeps up: the backlog left at the
    last arrival drains within `drain_s` and the completion rate after the
    warm-up reaches 90% of the offered rate."""
    return res["drain_s"] <= drain_s and res["throughput_qps"] >= 0.9 * rate


def bisect_rate(evaluate, lo: float, hi: float, steps: int):
    """Largest rate in [lo, hi] for which evaluate(rate) holds, by bisection
    on a log scale (evaluate(lo) is assumed to hold)."""
    if evaluate(hi):
        return hi
    for _ in range(steps):
        mid = math.sqrt(lo * hi)
        if evaluate(mid):
            lo = mid
        else:
            hi = mid
    return lo


def serving_leg(pm, n_req, rate, n_max, warmup_s, random_pool, bisect_steps):
    reqs = serving_requests(n_req, rate, n_max, random_pool)
    out = run_stream(pm, reqs, warmup_s)
    out.update({"offered_rate_qps": rate, "warmup_s": warmup_s, "random_pool": random_pool,
                "mix": f"1/3 random QP (n log-uniform in [20, {n_max}], m = 10n, drawn from a "
                       f"pool of {random_pool}, each a fresh request), 1/3 MPC (64 plants, "
                       "repeats change x0), 1/3 portfolio (16 models, repeats change mu)"})
    if bisect_steps > 0:
        window = 2.0

        def ok(r):
            rq = serving_requests(int(r * (window + warmup_s)), r, n_max, random_pool,
                                  seed_index=1)
            res = run_stream(pm, rq, warmup_s)
            print(f"# serving rate {r:.0f}/s: {res['throughput_qps']} solved/s, "
                  f"drain {res['drain_s']} s", file=sys.stderr, flush=True)
            return sustainable(res, r)

        out["sustainable_rate_qps"] = round(bisect_rate(ok, 25.0, rate, bisect_steps), 1)
    return out


def workload_leg(pm, name, steps=3, warmup=1, sample=16, threads=16, count=None):
    """Another workload timed as the main one is (its batch, launch shape,
    kernel time from the batch's events, the algorithmic byte model), with
    its own CPU baseline: the oracle on `sample` QPs spread over the batch,
    whose results are also the reference of the error report."""
    qps, desc, extra = build_workload(name, count)
    t0 = time.perf_counter()
    batch = pm.Batch(qps, precision="fp32", **extra)
    setup_s = time.perf_counter() - t0
    try:
        shape = DEFAULT_SHAPES.get(name)
        if shape:
            batch.set_shape(*(int(v) for v in shape.split(":")))
        for _ in range(warmup):
            batch.reset()
            batch.solve()
        kernel_ms, t0 = [], time.perf_counter()
        for _ in range(steps):
            batch.reset()
            batch.solve()
            kernel_ms.append(batch.last_kernel_ms())
        ms = (time.perf_counter() - t0) * 1e3 / steps
        results = [batch.get(i) for i in range(len(qps))]
    finally:
        batch.close()
    infos = [r[2] for r in results]
    kms = float(np.mean(kernel_ms))
    algo = algorithmic_bytes(qps, infos)
    achieved = algo / (kms * 1e-3) / 1e9
    idx = sorted(set(np.linspace(0, len(qps) - 1, min(sample, len(qps))).astype(int).tolist()))
    sub = [qps[i] for i in idx]
    refs, cpu_wall = oracle_pool(sub, extra, min(threads, len(sub)))
    solved = sum(1 for i in infos if i["status_name"] == "solved")
    paths = {}
    for i in infos:
        paths[LINSYS_NAMES.get(i["linsys"], "?")] = paths.get(LINSYS_NAMES.get(i["linsys"], "?"), 0) + 1
    return {"workload": desc, "count": len(qps), "steps": steps, "setup_s": round(setup_s, 3),
            "ms_per_step": round(ms, 3), "solved": solved,
            "solved_qps_per_s": round(solved / (ms * 1e-3), 2), "linsys": paths,
            "mean_iter": round(float(np.mean([i["iter"] for i in infos])), 1),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": None, "kernel": KERNEL[name], "kernel_ms": round(kms, 3),
                         "algorithmic_bytes": algo},
            "error_vs_oracle": error_report(sub, [results[i] for i in idx], refs),
            "cpu_baseline": {"value": round(sum(r.status == "solved" for r in refs) / cpu_wall, 2),
                             "unit": "QPs/s", "cores": min(threads, len(sub)), "kind": "oracle",
                             "sample": f"{len(sub)} of {len(qps)} QPs spread over the batch"}}


LINSYS_NAMES = {1: "jacobi_pcg", 2: "dense", 3: "lowrank", 4: "band"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="portfolio", choices=sorted(WORKLOADS))
    ap.add_argument("--count", type=int, default=None, help="override the batch size")
    ap.add_argument("--fp64-budget", type=float, default=10.0)
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--serving-full", action="store_true",
                    help="the serving configuration: 20000 requests at 2000/s, n up to 5000, "
                         "first second discarded")
    ap.add_argument("--serving-requests", type=int, default=3000)
    ap.add_argument("--serving-rate", type=float, default=2000.0)
    ap.add_argument("--serving-nmax", type=int, default=1000,
                    help="largest random-QP n in the serving mix")
    ap.add_argument("--serving-warmup", type=float, default=1.0)
    ap.add_argument("--serving-pool", type=int, default=16,
                    help="distinct random QPs the fresh random requests are drawn from")
    ap.add_argument("--serving-bisect", type=int, default=0,
                    help="bisection steps for the sustainable rate (0: none)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-side-workloads", action="store_true",
                    help="skip the other workloads' legs (MPC batch, full-size Lasso)")
    ap.add_argument("--no-parametric", action="store_true")
    ap.add_argument("--no-high-accuracy", action="store_true")
    ap.add_argument("--shape", default=None,
                    help="BLOCK:LANE_DIV launch shape for the timed steps (default: the "
                         "workload's entry in DEFAULT_SHAPES; 'setup' keeps the setup's shape)")
    ap.add_argument("--graph", action="store_true",
                    help="solve through the replayable graph of the solve launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU run is not supported", file=sys.stderr)
        sys.exit(2)

    import paper_1711_08013_amd as pm
    if pm.device_count() < 1:
        print("bench.py: no HIP device visible", file=sys.stderr)
        sys.exit(1)

    qps, desc, extra = build_workload(args.workload, args.count)
    print(f"# workload {args.workload}: {len(qps)} QPs built", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    batch = pm.Batch(qps, precision="fp32", **extra)
    setup_s = time.perf_counter() - t0
    print(f"# setup {setup_s:.2f} s", file=sys.stderr, flush=True)
    shape = None
    shape_arg = args.shape if args.shape else DEFAULT_SHAPES.get(args.workload, "setup")
    if shape_arg != "setup":
        shape = tuple(int(v) for v in shape_arg.split(":"))
        batch.set_shape(*shape)

    def step():
        batch.reset()
        if args.graph:
            batch.solve_graph()
        else:
            batch.solve()

    for w in range(args.warmup):
        step()
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    kernel_ms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        kernel_ms.append(batch.last_kernel_ms())
        print(f"# step {k}: solve kernels {kernel_ms[-1]:.2f} ms", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    results = [batch.get(i) for i in range(len(qps))]
    infos = [r[2] for r in results]
    ms_per_step = elapsed * 1e3 / args.steps
    lat = np.array([i["solve_time"] for i in infos]) * 1e3
    statuses = {}
    for i in infos:
        statuses[i["status_name"]] = statuses.get(i["status_name"], 0) + 1

    algo = algorithmic_bytes(qps, infos)
    pbytes = path_bytes(qps, infos)
    kms = float(np.mean(kernel_ms))
    achieved = algo / (kms * 1e-3) / 1e9
    traffic = stored_traffic(args.workload, shape) if args.count is None else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL[args.workload], "kernel_ms": round(kms, 3),
                "algorithmic_bytes": algo,
                "path_bytes": pbytes,
                "path_gbs": round(pbytes / (kms * 1e-3) / 1e9, 1)}

    # the oracle on every QP of the batch, on a pool of host threads: the
    # CPU baseline and the reference each GPU result is checked against
    threads = host_threads()
    print(f"# oracle on {len(qps)} QPs, {threads} threads", file=sys.stderr, flush=True)
    refs, cpu_wall = oracle_pool(qps, extra, threads)
    errors = error_report(qps, results, refs)
    # solved = the GPU and the oracle both report "solved"
    solved = sum(1 for i, r in zip(infos, refs)
                 if i["status_name"] == "solved" and r.status == "solved")
    value = solved / (ms_per_step * 1e-3)
    cpu_solved = sum(1 for r in refs if r.status == "solved")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "QPs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": desc, "count": len(qps),
                                        "eps_abs": 1e-3, "eps_rel": 1e-3,
                                        "precision": "fp32 products/updates, fp64 residual "
                                                     "each step, fp64 checks",
                                        "polish": int(extra.get("polish", 0))},
        "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_latency_ms": round(float(np.percentile(lat, 99)), 3),
        "batch_latency_ms": round(ms_per_step, 3),
        "statuses": statuses, "setup_s": round(setup_s, 3),
        "launch": {"shape": list(shape) if shape else "setup", "graph": bool(args.graph)},
        "device": pm.device_info(),
        "roofline": roofline,
        "error_vs_oracle": errors,
        "cpu_baseline": {"value": round(cpu_solved / cpu_wall, 2), "unit": "QPs/s",
                         "cores": threads, "kind": "oracle",
                         "sample": f"all {len(qps)} QPs of the timed batch, one QP per task on "
                                   f"{threads} host threads ({cpu_wall:.1f} s wall)",
                         "nproc": os.cpu_count(), "cpu_model": cpu_model()},
    }
    batch.close()

    # the legs beside the metric: a failure in one is recorded in its entry
    # (with the exception) and the line is still printed
    def leg(name, fn):
        print(f"# {name}", file=sys.stderr, flush=True)
        try:
            out[name] = fn()
        except Exception as e:   # noqa: BLE001 -- reported, not hidden
            print(f"# {name} failed: {e!r}", file=sys.stderr, flush=True)
            out[name] = {"error": repr(e)}

    if not args.no_baselines:
        leg("fp64_plain", lambda: fp64_plain(pm, qps, args.fp64_budget, extra))
        f64 = out["fp64_plain"].get("qps", 0.0)
        out["speedup_vs_fp64_plain"] = round(value / f64, 2) if f64 > 0 else None
    if not args.no_high_accuracy:
        leg("high_accuracy", lambda: high_accuracy_leg(pm, qps, extra, shape))
    if not args.no_side_workloads:
        # the workloads not timed above, each with its own oracle sample
        others = {}
        for name in WORKLOADS:
            if name == args.workload:
                continue
            leg(f"workload_{name}", lambda name=name: workload_leg(pm, name, threads=threads))
            others[name] = out.pop(f"workload_{name}")
        out["other_workloads"] = others
    if not args.no_parametric:
        leg("parametric", lambda: parametric_leg(pm))
    if not args.no_serving:
        if args.serving_full:
            cfg = dict(SERVING_FULL)
            cfg["random_pool"] = max(args.serving_pool, 64)
        else:
            cfg = {"requests": args.serving_requests, "rate": args.serving_rate,
                   "n_max": args.serving_nmax, "warmup_s": args.serving_warmup,
                   "random_pool": args.serving_pool}

        def serving():
            res = serving_leg(pm, cfg["requests"], cfg["rate"], cfg["n_max"], cfg["warmup_s"],
                              cfg["random_pool"], args.serving_bisect)
            res["configuration"] = "full" if args.serving_full else "reduced"
            return res

        leg("serving", serving)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
