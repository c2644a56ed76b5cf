"""The library's kernels run on the CPU: the library source is built for the
host against a stand-in HIP runtime that executes every workgroup thread as
a fiber with wave-level shuffles, ballots and 16x16x4 matrix products
emulated (tests/simt), under the host address sanitizer.  The same C ABI
then solves the cases of tests/simt/runner.py -- every linear-system path
in both precisions, polishing (single QPs, and a batch in which a
workgroup polishes QPs of different shapes in turn), every launch shape
set_shape accepts, graph replays, the whole-grid team of a cooperative
launch, the serving loop, degenerate inputs, certificates, the appendix
problem classes and the parametric updates -- and each result is compared
with the oracle; the GPU edge-case and settings test files run against the
same build.  A device-memory access outside its allocation aborts the run
with the sanitizer's report, and a barrier or cross-lane operation that not
every thread reaches aborts it with the call sites.  This checks the
kernels' logic and indexing, not the GPU's timing or its hardware-specific
behaviour."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIMT = os.path.join(ROOT, "tests", "simt")


def _load_builder():
    import importlib.util
    spec = importlib.util.spec_from_file_location("simt_build", os.path.join(SIMT, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


simt_build = _load_builder()

# the runner's cases, split over four processes that run side by side
GROUPS = [["shapes"], ["grid"], ["graph", "paths", "mpc"], ["server_estimate"],
          ["polish", "polish_batch", "edges", "certificates", "appendix", "updates", "server",
           "allocator"]]
EXPECTED_OK = {"shapes": 1, "grid": 2, "graph": 1, "paths": 8, "mpc": 1, "polish": 4, "polish_batch": 2,
               "edges": 6,
               "certificates": 2, "appendix": 6, "updates": 1, "server": 2, "allocator": 1,
               "server_estimate": 6}


@pytest.fixture(scope="module")
def simt_lib():
    if not os.path.exists(simt_build.CLANG):
        pytest.skip("host clang++ not available")
    try:
        asan = simt_build.asan_runtime()
    except (RuntimeError, subprocess.CalledProcessError, FileNotFoundError):
        pytest.skip("address-sanitizer runtime not available")
    simt_build.build()
    return asan


# GPU test files run against the emulated kernels in the CPU suite, with
# the least number of tests each must hold
GPU_FILES_CPU = {"test_gpu_y_edge_cases.py": 21, "test_gpu_settings.py": 24}


def _finish(p, timeout):
    try:
        out, _ = p.communicate(timeout=timeout)
    except subprocess.TimeoutExpired:
        p.kill()
        out, _ = p.communicate()
    return p.returncode, out


@pytest.fixture(scope="module")
def emulated_runs(simt_lib):
    """The runner's case groups and the GPU test files above, all started
    at once (each is one process on the emulated kernels), then collected:
    {("runner", group index) | ("file", name): (return code, output)}."""
    env = dict(os.environ, LD_PRELOAD=simt_lib, ASAN_OPTIONS="detect_leaks=0",
               SIMT_WATCHDOG="300")
    procs = {}
    # the cooperative launch runs its whole grid (one workgroup per CU) side
    # by side: that group runs on an emulated device of three CUs
    for gi, g in enumerate(GROUPS):
        procs[("runner", gi)] = subprocess.Popen(
            [sys.executable, os.path.join(SIMT, "runner.py"), *g], stdout=subprocess.PIPE,
            stderr=subprocess.STDOUT, text=True,
            env=dict(env, SIMT_CUS="3") if g == ["grid"] else env, cwd=ROOT)
    for name in GPU_FILES_CPU:
        procs[("file", name)] = subprocess.Popen(
            [sys.executable, os.path.join(SIMT, "pytest_on_simt.py"),
             os.path.join(ROOT, "tests", name), "-m", "gpu", "-q"],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, cwd=ROOT)
    return {k: _finish(p, 900) for k, p in procs.items()}


def test_kernels_on_cpu_match_oracle(emulated_runs):
    outs = [v for k, v in emulated_runs.items() if k[0] == "runner"]
    text = "\n".join(o for _, o in outs)
    print(text)
    for rc, out in outs:
        assert rc == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in text
    for name, k in EXPECTED_OK.items():
        got = sum(1 for line in text.splitlines() if line.startswith(f"ok {name}:"))
        assert got == k, (name, got, k)


@pytest.mark.parametrize("name", sorted(GPU_FILES_CPU))
def test_gpu_file_runs_on_cpu_kernels(emulated_runs, name):
    """Two GPU test files with the emulated kernels in place of the device:
    the edge cases (degenerate inputs against closed forms, the oracle and
    the solve alone) and the settings sweep (the oracle's iteration counts on
    the exact paths)."""
    rc, out = emulated_runs[("file", name)]
    print(out[-3000:])
    assert rc == 0, out[-6000:]
    # every GPU test of the file ran and passed (none skipped)
    path = os.path.join(ROOT, "tests", name)
    c = subprocess.run([sys.executable, "-m", "pytest", "--collect-only", "-q", "-m", "gpu",
                        "-p", "no:cacheprovider", path],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    n = sum(1 for line in c.stdout.splitlines() if "::" in line)
    assert n >= GPU_FILES_CPU[name], c.stdout
    assert f"{n} passed" in out and "skipped" not in out, out[-500:]


# Every GPU test file against the emulated kernels: an hour or more per file,
# so only on request (OSQPMI_EMULATE_GPU_FILES=1).  The cases sized for the
# device alone (the full-size Lasso, the benchmark's full batches) are left
# out; the whole-grid tests (the batched file, polishing after the
# whole-grid team) run on three emulated CUs, where a whole-grid launch is
# 1,536 fibers instead of 131,072.
GPU_FILES = [
    ("test_gpu_parity.py", "not lasso_full_size and not whole_grid", None),
    ("test_gpu_parity.py", "whole_grid", "3"),
    ("test_gpu_batched.py", None, "3"),
    ("test_gpu_parametric.py", None, None),
    ("test_gpu_high_accuracy.py", None, None),
    ("test_gpu_serving.py", None, None),
    ("test_gpu_extra_workloads.py", None, None),
]


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("OSQPMI_EMULATE_GPU_FILES") != "1",
                    reason="hours of emulation; set OSQPMI_EMULATE_GPU_FILES=1")
@pytest.mark.parametrize("name,select,cus", GPU_FILES)
def test_gpu_file_on_cpu_kernels(simt_lib, name, select, cus):
    env = dict(os.environ, LD_PRELOAD=simt_lib, ASAN_OPTIONS="detect_leaks=0",
               SIMT_WATCHDOG="5000")
    if cus:
        env["SIMT_CUS"] = cus
    args = [sys.executable, os.path.join(SIMT, "pytest_on_simt.py"),
            os.path.join(ROOT, "tests", name), "-m", "gpu", "-q", "-p", "no:faulthandler"]
    if select:
        args += ["-k", select]
    r = subprocess.run(args, capture_output=True, text=True, env=env, cwd=ROOT, timeout=6 * 3600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert " passed" in r.stdout and "failed" not in r.stdout
