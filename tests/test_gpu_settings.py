"""The solver settings on the GPU, against the oracle: on the exact-factor
paths in FP64 (dense factor, band factor, low-rank form) every ADMM step is
the direct method's, so for each setting the device must take the oracle's
iteration count, rho-bar updates and status, and reach its objective to
FP64 rounding.  A setting the device read differently from the oracle (a
relaxation, a check period, a step size, a tolerance) shows as another
iteration count.  The time limit is checked on its own: the oracle's clock
is not the device's."""
from __future__ import annotations

import pytest

import oracle
import qpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import paper_1711_08013_amd as pm
    assert pm.device_count() > 0, "no HIP device"
    return pm


# one setting changed at a time from the defaults (Section 5.2's rho rule,
# the relaxation of Algorithm 1, the check period, the step sizes, Ruiz
# passes, the tolerances, the iteration cap)
SWEEP = [
    {}, {"check_every": 1}, {"check_every": 10}, {"alpha": 1.0}, {"alpha": 1.9},
    {"rho": 0.01}, {"rho": 1.0}, {"sigma": 1e-3}, {"adaptive_rho": 0},
    {"scaling_iters": 0}, {"scaling_iters": 3}, {"eps_abs": 1e-5, "eps_rel": 1e-5},
    {"max_iter": 60, "check_every": 7},
]
SHORT = [{"alpha": 1.0}, {"check_every": 10}, {"rho": 0.01}, {"adaptive_rho": 0}]


def _case(pm, qp, linsys, code, kw):
    ref = oracle.solve(qp, **kw)
    x, y, info = pm.solve(qp, precision="fp64", linsys=linsys, **kw)
    label = f"{qp.name} {linsys} {kw}"
    print(f"{label}: {info['status_name']} {info['iter']} iterations, "
          f"{info['rho_updates']} rho updates (oracle {ref.status} {ref.iter})", flush=True)
    assert info["linsys"] == code, label
    assert info["status_name"] == ref.status, label
    assert info["iter"] == ref.iter, label
    assert info["rho_updates"] == ref.rho_updates, label
    assert abs(info["obj_val"] - ref.obj_val) <= 1e-9 * max(1.0, abs(ref.obj_val)), label


@pytest.mark.parametrize("kw", SWEEP, ids=lambda kw: ",".join(f"{k}={v}" for k, v in kw.items())
                         or "defaults")
def test_dense_factor_follows_every_setting(pm, kw):
    _case(pm, qpgen.config_instance(1, 2), "dense", 2, kw)


@pytest.mark.parametrize("kw", SHORT, ids=lambda kw: ",".join(f"{k}={v}" for k, v in kw.items()))
def test_band_and_lowrank_follow_the_settings(pm, kw):
    _case(pm, qpgen.mpc(qpgen.rng_for(3, 7), T=12), "band", 4, kw)
    _case(pm, qpgen.config_instance(4, 2, n_range=(100, 101)), "lowrank", 3, kw)


def test_time_limit(pm):
    """A limit far below one check period stops the solve at the first check
    with "time_limit_reached"; a generous one changes nothing."""
    qp = qpgen.config_instance(1, 2)
    _, _, info = pm.solve(qp, precision="fp64", time_limit=1e-9)
    assert info["status_name"] == "time_limit_reached" and info["iter"] == 25
    _, _, info = pm.solve(qp, precision="fp64", time_limit=100.0)
    assert info["status_name"] == "solved" and info["iter"] == oracle.solve(qp).iter


def _infeasible_pair():
    """A random QP made primal infeasible by one row bounded below by 1 and
    the same row bounded above by -1; and one made dual infeasible by taking
    variable 0 out of P and A, giving it q_0 = -1 and only the bound x_0 >= 0
    (the ray e_0 lowers the objective without end)."""
    import numpy as np
    import scipy.sparse as sp
    from qpgen import QP
    base = qpgen.random_qp(20, qpgen.rng_for(9, 40))
    a = np.random.default_rng(3).standard_normal(20)
    A = sp.vstack([base.A, sp.csr_matrix(a), sp.csr_matrix(a)], format="csr")
    pinf = QP(base.P, base.q, A, np.concatenate([base.l, [1.0, -np.inf]]),
              np.concatenate([base.u, [np.inf, -1.0]]), name="primal infeasible")
    Pd = base.full_P().toarray()
    Pd[0, :] = 0.0
    Pd[:, 0] = 0.0
    Ad = base.A.toarray()
    Ad[:, 0] = 0.0
    Ad = np.vstack([Ad, np.eye(20)[:1]])
    dinf = QP(sp.csr_matrix(np.triu(Pd)), np.concatenate([[-1.0], base.q[1:]]), sp.csr_matrix(Ad),
              np.concatenate([base.l, [0.0]]), np.concatenate([base.u, [np.inf]]),
              name="dual infeasible")
    return pinf, dinf


@pytest.mark.parametrize("eps_inf", [1e-4, 1e-6, 1e-2])
def test_certificates_follow_the_tolerances(pm, eps_inf):
    """The infeasibility tests of Section 3.4 with their tolerances changed:
    on the FP64 dense factor each certificate is found at the check where
    the oracle finds it (the iteration count moves with the tolerance)."""
    for qp in _infeasible_pair():
        ref = oracle.solve(qp, eps_pinf=eps_inf, eps_dinf=eps_inf)
        x, y, info = pm.solve(qp, precision="fp64", linsys="dense", eps_prim_inf=eps_inf,
                              eps_dual_inf=eps_inf)
        label = f"{qp.name} eps_inf={eps_inf}"
        print(f"{label}: {info['status_name']} at {info['iter']} (oracle {ref.status} at "
              f"{ref.iter})", flush=True)
        assert info["status_name"] == ref.status == qp.name.replace(" ", "_"), label
        assert info["iter"] == ref.iter and info["rho_updates"] == ref.rho_updates, label


@pytest.mark.parametrize("kw", [{}, {"delta": 1e-8}, {"polish_refine_iter": 0}],
                         ids=["defaults", "delta=1e-8", "no_refinement"])
def test_polish_follows_its_settings(pm, kw):
    """Polishing (Section 4) with its regularisation and its refinement count
    changed, after the FP64 solve on the dense, low-rank and band paths: the
    device accepts or rejects the polished point as the oracle does, and an
    accepted point is the oracle's (x to 1e-8, the objective to 1e-9)."""
    import numpy as np
    for qp in (qpgen.config_instance(1, 2), qpgen.config_instance(4, 3, n_range=(100, 101)),
               qpgen.mpc(qpgen.rng_for(3, 7), T=12)):
        ref = oracle.solve(qp, polish=1, **kw)
        x, y, info = pm.solve(qp, precision="fp64", polish=1, **kw)
        label = f"{qp.name} {kw}"
        print(f"{label}: polish {info['polish_status']} (oracle {ref.polish_status})", flush=True)
        assert info["status_name"] == ref.status == "solved", label
        assert info["polish_status"] == ref.polish_status, label
        if ref.polish_status == 1:
            assert np.max(np.abs(x - ref.x)) <= 1e-8 * max(1.0, np.max(np.abs(ref.x))), label
            assert abs(info["obj_val"] - ref.obj_val) <= 1e-9 * max(1.0, abs(ref.obj_val)), label
