"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the two byte
models (the algorithmic bytes of the method and the bytes of this
implementation's passes) on a hand-counted instance, the rule that ties the
stored counter traffic to the kernel sources and the launch shape, the error
report against the oracle, the serving statistics and the rate bisection."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import scipy.sparse as sp

import bench
from qpgen import QP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _tiny():
    # n = 3, m = 4; A rows: 2 entries, 1, 3, 1 -> a = 7, multi-entry rows R = 2
    # holding a_m = 5 entries; P upper: diagonal 3 + one off-diagonal -> full 5
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0],
                                [0.0, 1.0, 0.0],
                                [1.0, 1.0, 1.0],
                                [0.0, 0.0, 4.0]]))
    P = sp.csr_matrix(np.array([[2.0, 1.0, 0.0],
                                [0.0, 2.0, 0.0],
                                [0.0, 0.0, 1.0]]))
    return QP(P, np.zeros(3), A, -np.ones(4), np.ones(4), name="tiny")


def test_algorithmic_bytes_hand_count():
    """Per PCG iteration 16a + 8p + 4(12n + 4m); per ADMM step one more such
    pass plus 4(5n + 12m); per check 12(2a + p) + 8(6n + 6m); no factor."""
    qp = _tiny()
    n, m, a, p = 3, 4, 7, 5
    pcg_b = 16 * a + 8 * p + 4 * (12 * n + 4 * m)          # 112 + 40 + 208 = 360
    assert pcg_b == 360
    for path in (1, 2, 3):
        info = {"iter": 50, "pcg_iter": 80, "rho_updates": 1, "linsys": path}
        want = (80 + 50) * 360 + 50 * 4 * (5 * n + 12 * m) + 2 * (12 * (2 * a + p) + 8 * (6 * n + 6 * m))
        assert bench.algorithmic_bytes([qp], [info]) == want
    info = {"iter": 26, "pcg_iter": 26, "rho_updates": 0, "linsys": 3}
    assert bench.s8d_bytes(qp, info) == 52 * 360 + 26 * 4 * 63 + 2 * (12 * 19 + 8 * 42)


def test_path_bytes_hand_count():
    qp = _tiny()
    n, m, a, p, am, R = 3, 4, 7, 5, 5, 2
    e = 8                              # FP32 value + int32 index
    it, pcg, rho_up = 50, 80, 1
    admm = it * (e * (a + p) + 8 * (6 * n + m) + e * a + 8 * (3 * n + 9 * m))
    chk = 2 * (12 * (2 * a + p) + 8 * (6 * n + 6 * m))      # 50 / 25 checks
    pcg_b = e * (2 * a + p) + 4 * (2 * n + m) + 4 * (5 * n + 2 * m) + 16 * n
    # Jacobi: PCG products only
    info = {"iter": it, "pcg_iter": pcg, "rho_updates": rho_up, "linsys": 1}
    assert bench.path_bytes([qp], [info]) == admm + pcg * pcg_b + chk
    # dense factor: applies once per ADMM step and per extra inner step
    info["linsys"] = 2
    applies = (it + (pcg - it)) * (4 * n * n + 8 * n)
    fact = (1 + rho_up) * 3 * 4 * n * n
    assert bench.path_bytes([qp], [info]) == admm + pcg * pcg_b + applies + chk + fact
    # FP64 dense factor: the direct step, one apply per iteration
    info64 = {"iter": it, "pcg_iter": it, "rho_updates": rho_up, "linsys": 2}
    admm64 = it * (12 * (a + p) + 8 * (6 * n + m) + 12 * a + 8 * (3 * n + 9 * m))
    assert bench.path_bytes([qp], [info64], value_bytes=8) == \
        admm64 + it * (8 * n * n + 16 * n) + chk + (1 + rho_up) * 3 * 8 * n * n
    # low-rank direct step: one apply per counted inner step, no PCG products
    info["linsys"] = 3
    work = pcg * (e * (am + a) + 8 * (R * R + 4 * n + 2 * m))
    fact = (1 + rho_up) * (8 * (2 * R * n + R * R) + e * am)
    assert bench.path_bytes([qp], [info]) == admm + work + chk + fact
    # band direct step: one sweep pair over the FP64 tiles per counted step
    info["linsys"] = 4
    work = pcg * (16 * 64 * n + 24 * n)
    fact = (1 + rho_up) * (16 * 64 * n + e * (a + p))
    assert bench.path_bytes([qp], [info]) == admm + work + chk + fact


def test_stored_traffic_needs_matching_sources_and_shape(monkeypatch, tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "solve_wg_kernel_demo1024_traffic.md").write_text(
        "traffic_bytes_per_launch = 1.5e11\n"
        "kernel_source_sha256 = abc\n"
        "launch_shape = 512:32\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "abc")
    assert bench.stored_traffic("demo", (512, 32)) == 1.5e11
    assert bench.stored_traffic("demo", (256, 32)) is None
    assert bench.stored_traffic("demo", None) is None
    assert bench.stored_traffic("other", (512, 32)) is None
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "def")
    assert bench.stored_traffic("demo", (512, 32)) is None


def test_kernel_hash_covers_the_device_headers():
    csrc = os.path.join(ROOT, "paper_1711_08013_amd", "csrc")
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(csrc, f)), f
    # every local header the kernels include, directly or not, is hashed
    seen, todo = set(), ["kernels.h"]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            todo += [l.split('"')[1] for l in fh if l.startswith('#include "')]
    assert seen <= set(bench.KERNEL_SOURCES), seen - set(bench.KERNEL_SOURCES)


def test_error_report_against_oracle():
    """Status match, objective error, eps-scaled residuals and the x error
    (P diagonal and positive here) computed from the results as returned."""
    import oracle
    import qpgen
    qps = [qpgen.box_qp(np.array([1.0, 2.0]), np.array([-1.0, 1.0]), -np.ones(2), np.ones(2))
           for _ in range(3)]
    refs = [oracle.solve(q) for q in qps]
    good = (refs[0].x, refs[0].y, {"status_name": "solved", "obj_val": refs[0].obj_val})
    off = (refs[1].x + 1e-2, refs[1].y, {"status_name": "solved", "obj_val": refs[1].obj_val * 1.01})
    wrong = (refs[2].x, refs[2].y, {"status_name": "max_iter_reached", "obj_val": 0.0})
    rep = bench.error_report(qps, [good, off, wrong], refs)
    assert rep["status_match"] == 2 and rep["both_solved"] == 2
    assert abs(rep["max_rel_obj_err"] - 0.01 * abs(refs[1].obj_val) / max(1.0, abs(refs[1].obj_val))) < 1e-12
    assert rep["obj_err_above_1e-3"] == 1
    assert abs(rep["max_rel_x_err_p_definite"] - 1e-2 / max(1.0, np.max(np.abs(refs[1].x)))) < 1e-12
    # the perturbed point leaves the box by 1e-2: it fails the eps test
    assert rep["max_eps_scaled_prim"] > 1.0
    rep = bench.error_report(qps[:1], [good], refs[:1])
    assert rep["max_eps_scaled_prim"] <= 1.0 + 1e-9 and rep["max_eps_scaled_dual"] <= 1.0 + 1e-9


def test_latency_order_statistics_skip_warmup():
    arrivals = [0.1, 0.5, 1.0, 1.2, 1.5, 2.0]
    lats = [9.0, 9.0, 0.001, 0.002, 0.003, 0.004]
    st = bench.latency_stats(arrivals, lats, warmup_s=1.0)
    assert st["counted"] == 4
    assert st["p50_ms"] == 2.0          # 2nd of 4 (ceil(0.5 * 4) = 2)
    assert st["p99_ms"] == 4.0          # 4th of 4
    assert bench.latency_stats(arrivals, lats, warmup_s=5.0) is None


def test_sustainable_rate_bisection():
    calls = []

    def ok(r):
        calls.append(r)
        return r <= 300.0

    r = bench.bisect_rate(ok, 25.0, 2000.0, 12)
    assert 290.0 <= r <= 300.0 and calls[0] == 2000.0
    assert bench.bisect_rate(lambda r: True, 25.0, 2000.0, 5) == 2000.0
    assert bench.sustainable({"drain_s": 0.2, "throughput_qps": 950.0}, 1000.0)
    assert not bench.sustainable({"drain_s": 2.0, "throughput_qps": 950.0}, 1000.0)
    assert not bench.sustainable({"drain_s": 0.2, "throughput_qps": 500.0}, 1000.0)


def test_host_threads_capped():
    assert 1 <= bench.host_threads() <= 16
    assert bench.host_threads(cap=2) <= 2
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_every_workload_names_its_kernel():
    """Each workload the benchmark can time (the main one or a side leg)
    names the kernel its roofline divides by; the single large QP runs on
    the whole-grid kernel, the batches on the workgroup kernel."""
    assert set(bench.KERNEL) == set(bench.WORKLOADS)
    assert bench.WORKLOADS["lasso"][1] == 1 and bench.KERNEL["lasso"].startswith("solve_grid")
    for name in ("portfolio", "mpc"):
        assert bench.KERNEL[name].startswith("solve_wg")
