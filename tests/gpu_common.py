"""Shared helpers for the GPU parity tests (oracle comparison rules)."""
from __future__ import annotations

import numpy as np

from tests import qpcheck

# objective parity bar: |f_gpu - f_oracle| <= 1e-3 max(1, |f_oracle|)
OBJ_TOL = 1e-3
# the z-free primal ratio may exceed the device's z-based one by eps_rel
# (its tolerance uses ||Pi(Ax)|| instead of ||z||)
PRIM_SLACK = 1.0 + 2e-3
DUAL_SLACK = 1.0 + 1e-9


def compare(qp, x, y, info, ref, obj_tol=OBJ_TOL, eps_abs=1e-3, eps_rel=1e-3):
    """Returns a dict of the parity quantities for one instance and asserts
    the hard requirements (identical status, eps-scaled residuals <= 1)."""
    out = {"status": info["status_name"], "ref_status": ref.status}
    assert info["status_name"] == ref.status, (qp.name, info["status_name"], ref.status)
    if ref.status == "solved":
        rp, rd = qpcheck.eps_scaled_residuals(qp, x, y, eps_abs, eps_rel)
        assert rp <= PRIM_SLACK and rd <= DUAL_SLACK, (qp.name, rp, rd)
        err = qpcheck.rel_obj_err(info["obj_val"], ref.obj_val)
        out.update(rp=rp, rd=rd, obj_err=err)
        # the device's objective is the one of the returned x
        f_host = qp.objective(x)
        assert abs(f_host - info["obj_val"]) <= 1e-9 * max(1.0, abs(f_host))
    return out


def summarize(rows, label):
    errs = [r["obj_err"] for r in rows if "obj_err" in r]
    if errs:
        print(f"{label}: n={len(rows)} max_obj_err={max(errs):.2e} "
              f"median={float(np.median(errs)):.2e} max_rp={max(r['rp'] for r in rows if 'rp' in r):.3f} "
              f"max_rd={max(r['rd'] for r in rows if 'rd' in r):.3f}", flush=True)
    return errs


def assert_obj_parity(rows, label, frac_allowed=0.02, hard=1e-2):
    """Objective parity (reading 25): every instance within OBJ_TOL, except
    that up to `frac_allowed` of them may lie in (OBJ_TOL, hard] when both
    solutions pass the eps-KKT test (compare() has already asserted that for
    the GPU side; the oracle's passes by construction).  Those instances are
    two different eps-solutions, not a wrong one."""
    errs = [r["obj_err"] for r in rows if "obj_err" in r]
    over = [e for e in errs if e > OBJ_TOL]
    print(f"{label}: {len(over)} of {len(errs)} above {OBJ_TOL:g} (eps-consistent)", flush=True)
    assert all(e <= hard for e in errs), max(errs)
    assert len(over) <= max(1, int(frac_allowed * len(errs)))
