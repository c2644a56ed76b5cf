"""Runs pytest with the package bound to the host build of the library
(kernels on the CPU), so that a GPU test file's checks run against the
emulated kernels:
    python tests/simt/pytest_on_simt.py tests/test_gpu_y_edge_cases.py -m gpu
Started by the CPU test in a process of its own, with the sanitizer runtime
preloaded."""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import runner  # noqa: E402

if __name__ == "__main__":
    runner.load()
    import pytest
    sys.exit(pytest.main([*sys.argv[1:], "-p", "no:cacheprovider"]))
