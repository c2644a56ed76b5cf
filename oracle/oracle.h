/*
 * FP64 CPU oracle for the operator-splitting (ADMM) QP method of
 * Stellato et al., "OSQP: An Operator Splitting Solver for Quadratic Programs".
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the plain, slow reference that the
 * GPU path is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never does,
 * and the two share no code, header, table or helper.
 *
 * Problem:  minimize 1/2 x'Px + q'x  subject to  l <= Ax <= u   (Section 1, eq. pb:qp)
 * with P given as its upper triangle (diagonal included) in CSR, A in CSR.
 * Infinite bounds are IEEE inf; |b| >= 1e30 is also treated as infinite.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_SOLVED = 1,
  ORC_PRIMAL_INFEASIBLE = 2,
  ORC_DUAL_INFEASIBLE = 3,
  ORC_MAX_ITER_REACHED = 4,
  ORC_TIME_LIMIT_REACHED = 5,
  ORC_UNSOLVED = 6
};

typedef struct {
  int n, m;
  const int *P_indptr, *P_indices; const double *P_data;   /* upper triangle, CSR */
  const double *q;
  const int *A_indptr, *A_indices; const double *A_data;   /* m x n, CSR */
  const double *l, *u;
} orc_problem;

typedef struct {
  double rho, sigma, alpha, eps_abs, eps_rel, eps_pinf, eps_dinf, delta, time_limit;
  int max_iter, check_every, scaling_iters, adaptive_rho, polish, polish_refine_iter;
} orc_settings;

typedef struct {
  int status, iter, rho_updates, polish_status;  /* polish: 1 ok, -1 rejected, 0 not run */
  double obj_val, prim_res, dual_res, eps_prim, eps_dual, rho_bar;
  double setup_time, solve_time, polish_time;
} orc_info;

void orc_default_settings(orc_settings *s);

/* Full solve.  x_ws / y_ws (may be NULL) warm start in unscaled space.
 * Outputs x (n), y (m), z (m) in unscaled space.  Returns 0 or a negative
 * code on an internal failure (zero pivot, allocation). */
int orc_solve(const orc_problem *pb, const orc_settings *s,
              const double *x_ws, const double *y_ws,
              double *x, double *y, double *z, orc_info *info);

/* Section 5.2 rho-bar rule on scaled residuals and their normalisers (the
 * solver applies it at every termination check): returns the new rho-bar, or
 * rho_bar unchanged when the rule does not fire. */
double orc_rho_update(double rho_bar, double prim_res, double prim_norm, double dual_res,
                      double dual_norm);

/* Modified Ruiz equilibration alone: D (n), E (m), *c. */
int orc_ruiz(const orc_problem *pb, int iters, double *D, double *E, double *c);

/* Factor a symmetric quasi-definite matrix given as its upper triangle in CSC
 * (N x N) with LDL' after a minimum-degree ordering, then solve K x = b. */
int orc_ldl_solve(int N, const int *Kp, const int *Ki, const double *Kx,
                  const double *b, double *x);

/* The minimum-degree permutation used by the factorization (perm[k] = old index). */
int orc_mindeg(int N, const int *Kp, const int *Ki, int *perm);

#ifdef __cplusplus
}
#endif
#endif
