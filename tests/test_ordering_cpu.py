"""The host-side symbolic step of the band factor (csrc/ordering.h), on the
CPU: the reverse Cuthill-McKee ordering of the pattern of P + A'A returns a
permutation, the half-bandwidth it reports is the one numpy measures on the
reordered pattern, the MPC workload's reduced matrices come out within the
band the device factor accepts, and a row of A longer than the limit is
refused."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_08013_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "ordering.h"
// reads n m nnzP nnzA, then P's upper-triangle CSR and A's CSR (int32),
// prints the half-bandwidth and the permutation
int main(int argc, char **argv) {
  FILE *f = std::fopen(argv[1], "rb");
  int hdr[4];
  if (!f || std::fread(hdr, 4, 4, f) != 4) return 2;
  const int n = hdr[0], m = hdr[1], pn = hdr[2], an = hdr[3];
  std::vector<int> pp(n + 1), pi(pn), ap(m + 1), ai(an);
  if (std::fread(pp.data(), 4, n + 1, f) != (size_t)(n + 1) ||
      std::fread(pi.data(), 4, pn, f) != (size_t)pn ||
      std::fread(ap.data(), 4, m + 1, f) != (size_t)(m + 1) ||
      std::fread(ai.data(), 4, an, f) != (size_t)an) return 2;
  osqp_problem p{};
  p.n = n; p.m = m;
  p.P_upper = {n, n, pn, pp.data(), pi.data(), nullptr};
  p.A = {m, n, an, ap.data(), ai.data(), nullptr};
  std::vector<int> perm;
  const int bw = osqpmi::rcm_ordering(p, std::atoi(argv[2]), perm);
  std::printf("%d\n", bw);
  for (int v : perm) std::printf("%d ", v);
  std::printf("\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("ordering")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", CSRC, "-o", str(exe), str(src)])
    return d, exe


def _order(driver, qp, max_row=65):
    d, exe = driver
    P = sp.triu(qp.P).tocsr()
    A = qp.A.tocsr()
    fn = d / "qp.bin"
    with open(fn, "wb") as fh:
        np.array([qp.n, qp.m, P.nnz, A.nnz], np.int32).tofile(fh)
        for a in (P.indptr, P.indices, A.indptr, A.indices):
            np.asarray(a, np.int32).tofile(fh)
    out = subprocess.run([str(exe), str(fn), str(max_row)], capture_output=True, text=True,
                         check=True).stdout.split("\n")
    bw = int(out[0])
    perm = np.array([int(v) for v in out[1].split()], dtype=np.int64) if out[1].strip() else None
    return bw, perm


def _bandwidth(qp, perm):
    K = (abs(qp.full_P()) + abs(qp.A.T) @ abs(qp.A)).tocsr()
    K.setdiag(0)
    pos = np.empty(qp.n, dtype=np.int64)
    pos[perm] = np.arange(qp.n)
    C = K.tocoo()
    return int(np.max(np.abs(pos[C.row] - pos[C.col]))) if C.nnz else 0


@pytest.mark.parametrize("i", range(6))
def test_mpc_ordering_is_a_permutation_within_the_band(driver, i):
    qp = qpgen.config_instance(3, i)
    bw, perm = _order(driver, qp)
    assert sorted(perm.tolist()) == list(range(qp.n))
    assert bw == _bandwidth(qp, perm)
    # stage coupling: x_t, u_t, x_{t+1} -> 49 here, at most 64 accepted
    assert bw <= 56, bw


def test_chain_and_disconnected_patterns(driver):
    rng = np.random.default_rng(3)
    n = 60
    perm0 = rng.permutation(n)          # a chain hidden behind a random numbering
    rows = [[perm0[k], perm0[k + 1]] for k in range(n - 1)]
    A = sp.lil_matrix((n - 1, n))
    for r, (a, b) in enumerate(rows):
        A[r, a], A[r, b] = 1.0, -1.0
    qp = qpgen.QP(sp.csr_matrix(sp.identity(n)), np.zeros(n), A.tocsr(), -np.ones(n - 1),
                  np.ones(n - 1))
    bw, perm = _order(driver, qp)
    assert sorted(perm.tolist()) == list(range(n))
    assert bw == 1 == _bandwidth(qp, perm)
    # no coupling at all: every variable its own component, bandwidth 0
    qp0 = qpgen.QP(sp.csr_matrix(sp.identity(n)), np.zeros(n), sp.csr_matrix((0, n)),
                   np.zeros(0), np.zeros(0))
    bw, perm = _order(driver, qp0)
    assert bw == 0 and sorted(perm.tolist()) == list(range(n))


def test_long_row_is_refused(driver):
    qp = qpgen.config_instance(4, 0, n_range=(100, 101))   # the dense row 1'x = 1
    bw, _ = _order(driver, qp, max_row=65)
    assert bw == -1


@pytest.mark.parametrize("n,w", [(8192, 64), (8192, 56), (1000, 64)])
def test_banded_pattern_keeps_its_bandwidth(driver, n, w):
    """Windows of w + 1 consecutive variables (half-bandwidth w in the
    natural order): the ordering finds no narrower band and no wider one, so
    at n = 8192, w = 64 the device factor takes its largest block (64) and
    the permuted vector fills the solve's LDS stage exactly."""
    qp = qpgen.banded(np.random.default_rng(5), n, w)
    bw, perm = _order(driver, qp)
    assert sorted(perm.tolist()) == list(range(n))
    assert bw == w == _bandwidth(qp, perm)
    # the rows hold w + 1 entries: one more than the limit refuses them
    assert _order(driver, qp, max_row=w)[0] == -1
