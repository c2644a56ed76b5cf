"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the byte model
of the solve kernel on a hand-counted instance, and the rule that ties the
stored counter traffic to the kernel sources and the launch shape."""
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


def test_byte_model_hand_count():
    qp = _tiny()
    n, m, a, p, am, R = 3, 4, 7, 5, 5, 2
    e = 8                              # FP32 value + int32 index
    it, pcg, rho_up = 50, 80, 1
    admm = it * (e * (a + p) + 8 * (6 * n + m) + e * a + 8 * (3 * n + 9 * m))
    chk = 2 * (12 * (2 * a + p) + 8 * (6 * n + 6 * m))      # 50 / 25 checks
    pcg_b = e * (2 * a + p) + 4 * (2 * n + m) + 4 * (5 * n + 2 * m) + 16 * n
    # Jacobi: PCG products only
    info = {"iter": it, "pcg_iter": pcg, "rho_updates": rho_up, "linsys": 1}
    assert bench.algorithmic_bytes([qp], [info]) == admm + pcg * pcg_b + chk
    # dense factor: applies once per ADMM step and per extra inner step
    info["linsys"] = 2
    applies = (it + (pcg - it)) * (4 * n * n + 8 * n)
    fact = (1 + rho_up) * 3 * 4 * n * n
    assert bench.algorithmic_bytes([qp], [info]) == admm + pcg * pcg_b + applies + chk + fact
    # low-rank direct step: one apply per counted inner step, no PCG products
    info["linsys"] = 3
    work = pcg * (e * (am + a) + 8 * (R * R + 4 * n + 2 * m))
    fact = (1 + rho_up) * (8 * (2 * R * n + R * R) + e * am)
    assert bench.algorithmic_bytes([qp], [info]) == admm + work + chk + fact


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
