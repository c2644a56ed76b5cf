#!/usr/bin/env python3
"""Benchmark of the batched FP32-mixed ADMM QP path on one MI355X.

A step is one pass of the whole hot path over one batch with the problem data
already resident in HBM: device-side Ruiz equilibration, rho vector and
Jacobi preconditioner, the ADMM iterations with their warm-started PCG
solves, FP64 termination / infeasibility checks and rho adaptation,
unscaling (and polishing when enabled), then the results copied to the host.

Prints one JSON line.  Only --gpus 1 is supported: the library drives a
single GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import qpgen  # noqa: E402

METRIC = "solved QPs/s + p99 latency at eps 1e-3, FP32 batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (cfg, count, description, extra settings)
    "portfolio": (4, 1024, "batched factor-model portfolio, 1024 QPs, n in [100,2000], "
                           "k=n/10, F 50% dense", {"polish": 1}),
    "mpc": (3, 4096, "batched linear MPC, 4096 QPs, nx=20, nu=10, T in [5,20]", {}),
}
# launch shape (workgroup size : lane divisor) applied before the timed
# steps: the fastest of the shapes timed earlier on each workload (the same
# workgroup size the setup picks, so the grid stays the setup's)
DEFAULT_SHAPES = {"portfolio": "512:32", "mpc": "256:32"}


def build_workload(name: str, count: int | None):
    cfg, n_default, desc, extra = WORKLOADS[name]
    count = n_default if count is None else count
    qps = [qpgen.config_instance(cfg, i) for i in range(count)]
    return qps, desc, extra


def algorithmic_bytes(qps, infos, value_bytes=4, check_every=25):
    """Bytes the solve kernel must move, summed over the batch: each matrix
    once per application, at the width the path reads it (index 4 B + value
    vb = `value_bytes` in the ADMM passes, FP64 8 B in the checks), each
    vector once per pass.  Per QP with a = nnz(A), p = nnz(P full), a_m the
    entries of the R rows of A with several entries, e = 4 + vb:
      ADMM iteration : start pass A', P -> e (a + p) + 8 (6n + m);
                       update pass A    -> e a + 8 (3n + 9m)
      low-rank path  : one direct apply per iteration (counted in pcg_iter)
                       -> e (a_m + a) + 8 (R^2 + 4n + 2m); no PCG products
      dense path     : PCG iterations e (2a + p) + 4 (2n + m) + vb (5n + 2m) + 16n,
                       applies (ADMM iterations + inner iterations beyond the
                       first) vb n^2 + 2 vb n
      Jacobi path    : PCG iterations as above, no applies
      check (FP64, every 25 iterations): 12 (2a + p) + 8 (6n + 6m)
      factorisation (1 + rho updates): low-rank 8 (2 R n + R^2) + e a_m;
                                       dense 3 vb n^2
    """
    vb = value_bytes
    e = 4 + vb
    total = 0.0
    for qp, info in zip(qps, infos):
        n, m = qp.n, qp.m
        a = qp.A.nnz
        p = 2 * qp.P.nnz - int((qp.P.diagonal() != 0).sum())
        rl = np.diff(qp.A.indptr)
        am = int(rl[rl >= 2].sum())
        R = int((rl >= 2).sum())
        it, pcg = info["iter"], info["pcg_iter"]
        admm = it * (e * (a + p) + 8 * (6 * n + m) + e * a + 8 * (3 * n + 9 * m))
        pcg_b = e * (2 * a + p) + 4 * (2 * n + m) + vb * (5 * n + 2 * m) + 16 * n
        path = info.get("linsys", 1)
        if path == 3:
            work = pcg * (e * (am + a) + 8 * (R * R + 4 * n + 2 * m))
            fact_b = 8 * (2 * R * n + R * R) + e * am
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


def cpu_baseline(qps, budget_s: float, extra: dict):
    """The FP64 CPU oracle as it stands, single-threaded, on the first QPs of
    the same workload until about `budget_s` seconds of work are done."""
    import oracle
    oracle.build() if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")) else None
    t0 = time.perf_counter()
    solved = 0
    done = 0
    for qp in qps:
        r = oracle.solve(qp, polish=int(extra.get("polish", 0)))
        done += 1
        solved += r.status == "solved"
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": solved / dt, "unit": "QPs/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} QPs of the same workload, solved one after another "
                      f"on one host thread ({dt:.1f} s)"}


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


def serving_leg(pm, n_req: int, rate: float, n_max_random: int, gen_budget_s: float):
    """Continuous-batching server under a Poisson stream mixing the random-QP,
    MPC and portfolio generators (repeats of an MPC plant or a portfolio
    model share a structure key: resident data, update_vectors + warm
    start).  Requests are generated first (bounded by gen_budget_s), then
    submitted at their arrival times; latency is the server's own
    submit-to-completion time."""
    trace = qpgen.serving_trace(n_req, rate)
    state, reqs = {}, []
    t0 = time.perf_counter()
    for r in trace:
        qp = qpgen.serving_request(r, state, n_range=(20, n_max_random))
        if r["key"] is None:
            key = 0
        else:
            key = (1000 if r["key"][0] == "mpc" else 2000) + int(r["key"][1])
        reqs.append((r["t"], qp, key))
        if time.perf_counter() - t0 > gen_budget_s:
            break
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
    lat = np.array([o[3] for o in outs]) * 1e3
    solved = sum(1 for o in outs if o[2]["status_name"] == "solved")
    return {"requests": len(reqs), "offered_rate_qps": rate,
            "arrival_span_s": round(reqs[-1][0], 3), "wall_s": round(wall, 3),
            "throughput_qps": round(solved / wall, 1), "solved": solved,
            "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_ms": round(float(np.percentile(lat, 99)), 3),
            "mix": f"1/3 random QP (n log-uniform in [20, {n_max_random}], m = 10n), "
                   "1/3 MPC (64 plants, repeats change x0), 1/3 portfolio (16 models, "
                   "repeats change mu)",
            "micro_batches": stats["batches"], "peak_inflight": stats["peak_inflight"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="portfolio", choices=sorted(WORKLOADS))
    ap.add_argument("--count", type=int, default=None, help="override the batch size")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--fp64-budget", type=float, default=10.0)
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=600)
    ap.add_argument("--serving-rate", type=float, default=2000.0)
    ap.add_argument("--serving-nmax", type=int, default=1000,
                    help="largest random-QP n in the serving mix")
    ap.add_argument("--no-serving", action="store_true")
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
    tuning = None
    shape_arg = args.shape if args.shape else DEFAULT_SHAPES.get(args.workload, "setup")
    if shape_arg != "setup":
        blk, div = (int(v) for v in shape_arg.split(":"))
        batch.set_shape(blk, div)
        tuning = {"block_size": blk, "lane_div": div, "applied": True}

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
    infos = [batch.get(i)[2] for i in range(len(qps))]
    solved = sum(1 for i in infos if i["status_name"] == "solved")
    ms_per_step = elapsed * 1e3 / args.steps
    value = solved / (ms_per_step * 1e-3)
    lat = np.array([i["solve_time"] for i in infos]) * 1e3
    statuses = {}
    for i in infos:
        statuses[i["status_name"]] = statuses.get(i["status_name"], 0) + 1

    algo = algorithmic_bytes(qps, infos)
    kms = float(np.mean(kernel_ms))
    achieved = algo / (kms * 1e-3) / 1e9
    shape = (tuning["block_size"], tuning["lane_div"]) if tuning else None
    traffic = stored_traffic(args.workload, shape) if args.count is None else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "solve_wg_kernel<float>", "kernel_ms": round(kms, 3),
                "algorithmic_bytes": algo}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "QPs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": desc, "count": len(qps),
                                        "eps_abs": 1e-3, "eps_rel": 1e-3,
                                        "precision": "fp32 PCG/updates, fp64 checks",
                                        "polish": int(extra.get("polish", 0))},
        "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_latency_ms": round(float(np.percentile(lat, 99)), 3),
        "batch_latency_ms": round(ms_per_step, 3),
        "statuses": statuses, "setup_s": round(setup_s, 3),
        "launch": {"tuning": tuning, "graph": bool(args.graph)},
        "roofline": roofline,
    }
    if not args.no_baselines:
        f64 = fp64_plain(pm, qps, args.fp64_budget, extra)
        out["fp64_plain"] = f64
        out["speedup_vs_fp64_plain"] = round(value / f64["qps"], 2) if f64["qps"] > 0 else None
        out["cpu_baseline"] = cpu_baseline(qps, args.cpu_budget, extra)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    batch.close()
    if not args.no_high_accuracy:
        # the same batch at the paper's high-accuracy setting, eps = 1e-5
        print("# high accuracy", file=sys.stderr, flush=True)
        hb = pm.Batch(qps, precision="fp32", eps_abs=1e-5, eps_rel=1e-5, max_iter=20000, **extra)
        if shape:
            hb.set_shape(*shape)
        hb.reset()
        t0 = time.perf_counter()
        hb.solve()
        hs = time.perf_counter() - t0
        hinf = [hb.get(i)[2] for i in range(len(qps))]
        hsolved = sum(1 for i in hinf if i["status_name"] == "solved")
        out["high_accuracy"] = {"eps": 1e-5, "solved": hsolved, "qps_per_s": round(hsolved / hs, 2),
                                "batch_ms": round(hs * 1e3, 3),
                                "mean_iter": round(float(np.mean([i["iter"] for i in hinf])), 1)}
        hb.close()
    if not args.no_parametric:
        print("# parametric re-solves", file=sys.stderr, flush=True)
        out["parametric"] = parametric_leg(pm)
    if not args.no_serving:
        print("# serving stream", file=sys.stderr, flush=True)
        out["serving"] = serving_leg(pm, args.serving_requests, args.serving_rate,
                                     args.serving_nmax, gen_budget_s=30.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
