"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of oracle.c (a dropped term, a wrong sign, an inverted
ratio, a mean taken as a maximum ...), builds that copy, and runs the pins
named for it against the copy; at least one of them must fail.  The source
text each case replaces must be present in oracle.c, so a rewrite of the
oracle cannot turn a case into a silent no-op.  CPU only."""
from __future__ import annotations

import os

import pytest

import oracle
from tests import test_oracle_pins as pins

ORACLE_SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# name: (text in oracle.c, its replacement, pins that must catch it as
# (function, keyword arguments))
MUTATIONS = {
    "cost_scaling_mean_as_max": (
        "    for (int j = 0; j < n; ++j) mean += coln[j];\n    mean /= (double)n;\n",
        "    for (int j = 0; j < n; ++j) mean = dmax(mean, coln[j]);\n",
        [(pins.test_ruiz_passes_hand_values, {"case": c}) for c in pins._read_ruiz_golden()]),
    "cost_scaling_unscaled_q": (
        "    double s = dmax(mean, norm_inf(n, w->q));",
        "    double s = dmax(mean, norm_inf(n, w->q) / (w->D[0] * w->c));",
        [(pins.test_ruiz_passes_hand_values, {"case": c}) for c in pins._read_ruiz_golden()]),
    "ruiz_delta_without_sqrt": (
        "      dx[j] = 1.0 / sqrt(v);",
        "      dx[j] = 1.0 / v;",
        [(pins.test_ruiz_passes_hand_values, {"case": c}) for c in pins._read_ruiz_golden()]),
    "rho_rule_inverted_ratio": (
        "  double ratio = (prim_res / prim_norm) / (dual_res / dual_norm);",
        "  double ratio = (dual_res / dual_norm) / (prim_res / prim_norm);",
        [(pins.test_rho_rule_hand_values, {"row": r}) for r in pins._read_rho_rule()]),
    "rho_rule_without_sqrt": (
        "  double rnew = rho_bar * sqrt(ratio);",
        "  double rnew = rho_bar * ratio;",
        [(pins.test_rho_rule_hand_values, {"row": r}) for r in pins._read_rho_rule()]),
    "rho_rule_swapped_normalisers": (
        "  double ratio = (prim_res / prim_norm) / (dual_res / dual_norm);",
        "  double ratio = (prim_res / dual_norm) / (dual_res / prim_norm);",
        [(pins.test_rho_rule_hand_values, {"row": r}) for r in pins._read_rho_rule()]),
    "rho_rule_strict_gate": (
        "  if (rnew >= 5.0 * rho_bar || rnew <= rho_bar / 5.0) return rnew;",
        "  if (rnew > 5.0 * rho_bar || rnew < rho_bar / 5.0) return rnew;",
        [(pins.test_rho_rule_hand_values, {"row": r}) for r in pins._read_rho_rule()]),
    "rho_rule_without_clamp": (
        "  rnew = dmin(dmax(rnew, 1e-6), 1e6);\n  if (rnew >= 5.0",
        "  if (rnew >= 5.0",
        [(pins.test_rho_rule_hand_values, {"row": r}) for r in pins._read_rho_rule()]),
    "rho_rule_dual_normaliser_without_q": (
        "  r->dual_norm_s = dmax(pxs, dmax(atys, qqs));",
        "  r->dual_norm_s = dmax(pxs, atys);",
        [(pins.test_rho_rule_inside_solve_1d, {})]),
    "relaxation_dropped": (
        "    for (int j = 0; j < n; ++j) xb[j] = alpha * sol[j] + (1.0 - alpha) * xb[j];",
        "    for (int j = 0; j < n; ++j) xb[j] = sol[j];",
        [(pins.test_relaxed_contraction_rate_1d, {"alpha": 1.6})]),
    "dual_residual_sign": (
        "    double rd = Px[j] + w->q[j] + Aty[j];",
        "    double rd = Px[j] + w->q[j] - Aty[j];",
        [(pins.test_reported_residuals_match_definition, {"cfg": 1, "idx": 2, "kw": {}})]),
    "rho_vector_without_equality_factor": (
        "    rho[i] = (l_in[i] == u_in[i]) ? 1e3 * rho_bar : rho_bar;",
        "    rho[i] = rho_bar;",
        [(pins.test_equality_qp_is_iterative_refinement, {"seed": 0})]),
    "polish_refinement_sign": (
        "      for (int k = 0; k < N; ++k) t[k] += dt[k];",
        "      for (int k = 0; k < N; ++k) t[k] -= dt[k];",
        [(pins.test_polish_matches_brute_force, {})]),
    "polish_sign_test_on_equality_rows": (
        "      if (w->l[i] == w->u[i]) continue;\n",
        "",
        [(pins.test_polish_accepts_a_sign_free_equality_dual, {})]),
    "dual_infeasibility_sign": (
        "  if (!(qdx < -w->c * tol)) return 0;",
        "  if (!(qdx > w->c * tol)) return 0;",
        [(pins.test_dual_infeasible_certificate, {})]),
}


@pytest.fixture(scope="module")
def source():
    with open(ORACLE_SRC) as fh:
        return fh.read()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(oracle_lib, source, tmp_path, name):
    old, new, checks = MUTATIONS[name]
    assert source.count(old) == 1, f"{name}: text to replace not found once in oracle.c"
    # the unmodified oracle passes the same pins
    for fn, kw in checks:
        fn(oracle_lib, **kw)
    src = tmp_path / "oracle_planted.c"
    src.write_text(source.replace(old, new))
    lib = oracle.build(str(src), str(tmp_path / "liboracle_planted.so"))
    failed = []
    with oracle.use_library(lib):
        for fn, kw in checks:
            try:
                fn(oracle, **kw)
            except (AssertionError, RuntimeError) as e:
                failed.append((fn.__name__, type(e).__name__))
    assert failed, f"planted mistake {name} passed every pin named for it"
