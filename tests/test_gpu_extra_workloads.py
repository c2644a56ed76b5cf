"""The remaining appendix problem classes on the GPU through the C ABI --
equality-constrained QPs, Huber fitting and support vector machines -- at
the default settings, each against the oracle: status, eps-scaled residuals
and objective for every instance.  The larger Huber instances (n > 2500,
and their x columns keep them out of the low-rank form) take the
Jacobi-preconditioned path."""
from __future__ import annotations

import pytest

import oracle
import qpgen
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    assert pm.device_count() > 0, "no HIP device"
    return pm


def _instances():
    return ([qpgen.eq_qp(n, qpgen.rng_for(6, i)) for i, n in enumerate((20, 40, 60, 80, 100, 150))] +
            [qpgen.huber(qpgen.rng_for(7, i), nf) for i, nf in enumerate((5, 10, 15, 20))] +
            [qpgen.svm(qpgen.rng_for(8, i), nf) for i, nf in enumerate((5, 10, 15, 20))])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_extra_workloads_match_oracle(pm, precision):
    qps = _instances()
    print(f"extra workloads {precision}: {len(qps)} QPs", flush=True)
    b = pm.Batch(qps, precision=precision)
    b.solve()
    res = [b.get(i) for i in range(len(qps))]
    b.close()
    rows = [gc.compare(q, *r, oracle.solve(q)) for q, r in zip(qps, res)]
    gc.summarize(rows, f"extra workloads {precision}")
    exact = [row for row, r in zip(rows, res) if r[2]["linsys"] in (2, 3)]
    print(f"  exact-factor paths: {len(exact)} of {len(rows)}", flush=True)
    assert len(exact) >= 10
    gc.assert_obj_parity(rows, f"extra workloads {precision}")
