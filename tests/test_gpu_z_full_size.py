"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: the whole batch is solved in one launch, every QP's returned
point is checked against the Section 3.4 test recomputed in FP64 on the host,
and a sample spread over the size range is compared with the oracle one QP
at a time."""
from __future__ import annotations

import numpy as np
import pytest

import bench
import oracle
import qpgen
from tests import gpu_common as gc
from tests import qpcheck

pytestmark = pytest.mark.gpu

SAMPLE = 16


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    assert pm.device_count() > 0, "no HIP device"
    return pm


def _bench_batch(pm, workload):
    """The benchmark's batch and launch: same generator, count, settings and
    launch shape."""
    cfg, count, _, extra = bench.WORKLOADS[workload]
    print(f"{workload}: generating {count} QPs", flush=True)
    qps = [qpgen.config_instance(cfg, i) for i in range(count)]
    b = pm.Batch(qps, precision="fp32", **extra)
    blk, div = (int(v) for v in bench.DEFAULT_SHAPES[workload].split(":"))
    b.set_shape(blk, div)
    b.reset()
    b.solve()
    res = [b.get(i) for i in range(count)]
    b.close()
    print(f"{workload}: solved on the device at shape {blk}:{div}", flush=True)
    return qps, res, extra


def _check_all_and_sample(qps, res, polish):
    statuses = {}
    worst_p = worst_d = 0.0
    for qp, (x, y, info) in zip(qps, res):
        statuses[info["status_name"]] = statuses.get(info["status_name"], 0) + 1
        if info["status_name"] == "solved":
            rp, rd = qpcheck.eps_scaled_residuals(qp, x, y)
            worst_p, worst_d = max(worst_p, rp), max(worst_d, rd)
    print(f"  statuses {statuses}; worst eps-scaled residuals {worst_p:.3f} {worst_d:.3f}",
          flush=True)
    assert statuses == {"solved": len(qps)}
    assert worst_p <= gc.PRIM_SLACK and worst_d <= gc.DUAL_SLACK
    # sample: every len/SAMPLE-th QP in order of size
    order = np.argsort([q.n for q in qps], kind="stable")
    rows = []
    for i in order[:: max(1, len(qps) // SAMPLE)]:
        qp, (x, y, info) = qps[i], res[i]
        ref = oracle.solve(qp, polish=polish)
        row = gc.compare(qp, x, y, info, ref)
        if polish and info["polish_status"] == 1 and ref.polish_status == 1:
            assert row["obj_err"] <= 1e-6, (qp.name, row["obj_err"])
        rows.append(row)
    return rows


def test_portfolio_1024_at_bench_launch(pm):
    """Factor-model portfolios, 1024 QPs, FP32 with FP64 polish."""
    qps, res, extra = _bench_batch(pm, "portfolio")
    rows = _check_all_and_sample(qps, res, polish=extra.get("polish", 0))
    gc.summarize(rows, f"portfolio x1024 sample of {len(rows)}")
    assert max(r["obj_err"] for r in rows) <= gc.OBJ_TOL


def test_mpc_4096_at_bench_launch(pm):
    """Linear MPC, 4096 QPs, FP32, no polish."""
    qps, res, extra = _bench_batch(pm, "mpc")
    rows = _check_all_and_sample(qps, res, polish=extra.get("polish", 0))
    gc.summarize(rows, f"mpc x4096 sample of {len(rows)}")
    gc.assert_obj_parity(rows, f"mpc x4096 sample of {len(rows)}")
