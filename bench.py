#!/usr/bin/env python3
"""Benchmark of the batched FP32-mixed ADMM QP path on one MI355X.

A step is one pass of the whole hot path over one batch with the problem data
already resident in HBM: device-side Ruiz equilibration, rho vector and
Jacobi preconditioner, the ADMM iterations with their warm-started PCG
solves, FP64 termination / infeasibility checks and rho adaptation,
unscaling (and polishing when enabled), then the results copied to the host.

Prints one JSON line (see the design doc for every field).  Only --gpus 1 is
supported: this build uses a single GPU.
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


def build_workload(name: str, count: int | None):
    cfg, n_default, desc, extra = WORKLOADS[name]
    count = n_default if count is None else count
    qps = [qpgen.config_instance(cfg, i) for i in range(count)]
    return qps, desc, extra


def algorithmic_bytes(qps, infos, check_every=25, value_bytes=4, index_bytes=4):
    """Bytes the method must move per solve, summed over the batch: every
    sparse matrix application reads its values and indices once, vectors are
    read/written once per pass.  Per QP with a = nnz(A), p = nnz(P full):
      PCG iteration  : A p, A'(R t), P p  -> 2a + p entries, vectors 12n + 4m
      ADMM iteration : start pass (A', P) + update pass (A) -> 2a + p entries,
                       vectors 10n + 16m
      check (FP64)   : A, A', P in double -> 2a + p entries at 8+4 bytes,
                       vectors 8 (4n + 4m)
    """
    e = value_bytes + index_bytes
    total = 0.0
    for qp, info in zip(qps, infos):
        n, m = qp.n, qp.m
        a = qp.A.nnz
        p = 2 * qp.P.nnz - int((qp.P.diagonal() != 0).sum())
        pcg = info["pcg_iter"] * (e * (2 * a + p) + 4 * (12 * n + 4 * m))
        admm = info["iter"] * (e * (2 * a + p) + 4 * (10 * n + 16 * m))
        checks = -(-info["iter"] // check_every)
        chk = checks * ((8 + index_bytes) * (2 * a + p) + 8 * (4 * n + 4 * m))
        total += pcg + admm + chk
    return total


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in DESIGN.md", file=sys.stderr)
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

    def step():
        batch.reset()
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
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
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
        "roofline": roofline,
    }
    if not args.no_baselines:
        f64 = fp64_plain(pm, qps, args.fp64_budget, extra)
        out["fp64_plain"] = f64
        out["speedup_vs_fp64_plain"] = round(value / f64["qps"], 2) if f64["qps"] > 0 else None
        out["cpu_baseline"] = cpu_baseline(qps, args.cpu_budget, extra)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    batch.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
