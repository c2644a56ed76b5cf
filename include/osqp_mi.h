/*
 * osqp_mi -- MI355X (gfx950) implementation of the operator-splitting QP
 * method of Stellato, Banjac, Goulart, Bemporad and Boyd, "OSQP: An Operator
 * Splitting Solver for Quadratic Programs".
 *
 *   minimize   1/2 x'Px + q'x
 *   subject to l <= Ax <= u                                   (Section 1, eq. pb:qp)
 *
 * C ABI.  Every input pointer is host memory, borrowed for the duration of
 * the call only (the library copies what it needs).  Outputs go to caller
 * buffers.  Every function returns 0 on success or one of the OSQP_ERR_*
 * codes below; no C++ exception crosses this boundary.  A handle is used by
 * one host thread at a time; all device work of a handle runs on the stream
 * given in the settings (NULL: the library's own stream).
 */
#ifndef OSQP_MI_H
#define OSQP_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t osqp_int;
typedef double osqp_float;

/* ---- error codes (returned by every function) ------------------------- */
#define OSQP_OK 0
#define OSQP_ERR_DIM 1            /* n <= 0, m < 0, sizes disagree          */
#define OSQP_ERR_CSR 2            /* bad indptr/indices (range, order)      */
#define OSQP_ERR_P_NOT_UPPER 3    /* P holds an entry below the diagonal    */
#define OSQP_ERR_DATA_NONFINITE 4 /* NaN/inf in P, A or q; NaN in l or u    */
#define OSQP_ERR_L_GT_U 5         /* some l_i > u_i                          */
#define OSQP_ERR_SETTINGS 6       /* sigma<=0, rho<=0, alpha not in (0,2), eps<0, ... */
#define OSQP_ERR_ALLOC 7          /* device or host allocation failed       */
#define OSQP_ERR_BUDGET 8         /* request larger than the server's HBM budget */
#define OSQP_ERR_DEVICE 9         /* a HIP call failed                      */
#define OSQP_ERR_NOT_SETUP 10     /* NULL handle or missing data            */
#define OSQP_ERR_INDEX 11         /* problem index / ticket out of range    */
#define OSQP_ERR_NO_DEVICE 12     /* no HIP device visible                   */
#define OSQP_ERR_UNSUPPORTED 13   /* operation not available for this batch  */

/* ---- solve status (info.status), Sections 3.3-3.4 --------------------- */
#define OSQP_SOLVED 1
#define OSQP_PRIMAL_INFEASIBLE 2  /* y holds the certificate c^-1 E dy (Section 5.1) */
#define OSQP_DUAL_INFEASIBLE 3    /* x holds the certificate D dx (Section 5.1)      */
#define OSQP_MAX_ITER_REACHED 4
#define OSQP_TIME_LIMIT_REACHED 5
#define OSQP_UNSOLVED 6

/* ---- settings enums ----------------------------------------------------- */
#define OSQP_PRECISION_FP64 0       /* every step in double                  */
#define OSQP_PRECISION_FP32_MIXED 1 /* SpMV/PCG/updates in float; scaling,
                                       checks, certificates, polish in double */
#define OSQP_LINSYS_AUTO 0          /* low-rank form (P diagonal, few multi-   */
                                    /* entry rows of A), else the band factor  */
                                    /* (half-bandwidth <= 64 after ordering),  */
                                    /* else the dense factor for n <= 2500,    */
                                    /* else Jacobi PCG                         */
#define OSQP_LINSYS_PCG 1           /* reduced system, Section 3.1 indirect   */
#define OSQP_LINSYS_DENSE 2         /* dense Cholesky of the reduced matrix   */
                                    /* (n <= 4096, else Jacobi PCG): the      */
                                    /* direct step in FP64, the exact PCG     */
                                    /* preconditioner in FP32                 */
#define OSQP_LINSYS_LOWRANK 3       /* P diagonal, few multi-entry rows of A:  */
                                    /* Woodbury form of the reduced matrix,    */
                                    /* else as AUTO (the same order as AUTO)   */
#define OSQP_LINSYS_BAND 4          /* block-tridiagonal Cholesky factor of    */
                                    /* the reduced matrix after a reverse      */
                                    /* Cuthill-McKee ordering (Section 3.1's   */
                                    /* direct method on the reduced system),   */
                                    /* where the half-bandwidth is <= 64 and   */
                                    /* n <= 8192, in preference to the low-   */
                                    /* rank form; else as AUTO                 */

/* Compressed sparse rows.  indptr has nrows+1 entries, indptr[0] = 0,
 * non-decreasing, indptr[nrows] = nnz; each row's column indices strictly
 * increase and lie in [0, ncols). */
typedef struct {
  osqp_int nrows, ncols, nnz;
  const osqp_int *indptr;
  const osqp_int *indices;
  const osqp_float *data;
} osqp_csr;

/* One QP: P is the upper triangle of the symmetric cost matrix (diagonal
 * included), n x n; A is m x n.  Bounds: IEEE inf or |b| >= 1e30 mean
 * "no bound" (Section 1: l_i in {-inf} u R, u_i in R u {+inf}). */
typedef struct {
  osqp_int n, m;
  osqp_csr P_upper;
  const osqp_float *q;   /* n */
  osqp_csr A;
  const osqp_float *l;   /* m */
  const osqp_float *u;   /* m */
} osqp_problem;

typedef struct {
  osqp_float rho;          /* rho-bar^0 (Section 5.2), default 0.1          */
  osqp_float sigma;        /* Section 5.2, default 1e-6                      */
  osqp_float alpha;        /* relaxation, (0,2), default 1.6                  */
  osqp_float eps_abs, eps_rel;            /* Section 3.4, default 1e-3       */
  osqp_float eps_prim_inf, eps_dual_inf;  /* Section 3.4, default 1e-4       */
  osqp_float delta;        /* polish regularisation (Section 4), 1e-6        */
  osqp_float time_limit;   /* seconds of solve time, 0 = none                */
  osqp_float pcg_tol_frac; /* inner PCG tolerance factor (Jacobi path),      */
                           /* default 1e-3                                   */
  osqp_int max_iter;       /* default 4000                                   */
  osqp_int check_every;    /* termination-check interval, default 25         */
  osqp_int scaling_iters;  /* Ruiz passes (Section 5.1), default 10          */
  osqp_int adaptive_rho;   /* Section 5.2 rho-bar rule, default 1            */
  osqp_int polish;         /* Section 4, default 0                           */
  osqp_int polish_refine_iter; /* iterative-refinement passes, default 3     */
  osqp_int precision;      /* OSQP_PRECISION_*, default FP32_MIXED          */
  osqp_int linsys;         /* OSQP_LINSYS_*, default AUTO                    */
  osqp_int pcg_max_iter;   /* PCG iterations per ADMM step, default 50       */
  osqp_int block_size;     /* threads per workgroup, 0 = chosen by size     */
                           /* (512 for long passes, else 256;               */
                           /* osqp_batch_set_shape may change it); else     */
                           /* fixed, a multiple of 64                       */
  void *stream;            /* hipStream_t to run on, NULL = own stream       */
} osqp_settings;

typedef struct {
  osqp_int status;         /* OSQP_SOLVED, ...                               */
  osqp_int iter;           /* ADMM iterations                                */
  osqp_int pcg_iter;       /* total inner PCG iterations (one per ADMM      */
                           /* iteration where the step is a direct one)     */
  osqp_int rho_updates;
  osqp_int polish_status;  /* 1 accepted, -1 rejected, 0 not run; accepted */
                           /* when the polished residuals are not larger   */
                           /* than the ADMM ones and the duals of active   */
                           /* inequality rows keep their signs (Section 4) */
  osqp_int linsys;         /* reduced-system path assigned at setup:         */
                           /* OSQP_LINSYS_PCG (Jacobi), _DENSE, _LOWRANK or  */
                           /* _BAND; a factorisation that meets a pivot     */
                           /* that is not positive (FP32 rounding) solves   */
                           /* with Jacobi PCG instead; it is tried again   */
                           /* when rho-bar changes and at the next solve    */
  osqp_float obj_val;      /* 1/2 x'Px + q'x on the original data (FP64)    */
  osqp_float prim_res, dual_res, eps_prim, eps_dual; /* unscaled, FP64, Sections 3.4/5.1 */
  osqp_float rho_bar;      /* final rho-bar                                  */
  osqp_float setup_time, solve_time, polish_time;   /* seconds              */
  /* device time of this QP's solve by phase (seconds): dense factorisation,
   * PCG (start pass and iterations), ADMM update pass, FP64 checks */
  osqp_float factor_time, pcg_time, update_time, check_time;
} osqp_info;

/* Outcome of osqp_batch_autotune (which is switched off, see there). */
typedef struct {
  osqp_int block_size;     /* threads per workgroup chosen                   */
  osqp_int lane_div;       /* lanes per row ~ mean row length / lane_div      */
  osqp_int trials;         /* launch shapes timed                            */
  osqp_float default_ms;   /* device time of a cold solve, setup shape       */
  osqp_float best_ms;      /* device time of a cold solve, chosen shape      */
} osqp_tuning;

typedef struct osqp_batch osqp_batch;
typedef struct osqp_batch osqp_solver;   /* a single QP is a batch of one */
typedef struct osqp_server osqp_server;

/* Fill *s with the defaults listed above (Section 7 defaults where the paper
 * gives them).  Returns OSQP_ERR_NOT_SETUP if s is NULL. */
osqp_int osqp_set_default_settings(osqp_settings *s);

/* Human-readable name of an error code (static storage). */
const char *osqp_error_string(osqp_int code);

/* Device memory for the handles created after this call comes from
 * alloc(bytes, ctx) and goes back through free_fn(ptr, ctx) -- for instance a
 * framework's caching allocator, so that the solver's memory is counted and
 * reused with the caller's own.  alloc returns device memory of the current
 * device, aligned to at least 256 bytes, or NULL on failure (the setup then
 * returns OSQP_ERR_ALLOC).  Both NULL restores hipMalloc / hipFree.  Each
 * handle keeps the pair it was created with until its cleanup, which waits
 * for the handle's stream before freeing.  Callable from any thread; calls
 * take effect for setups that start after them.  OSQP_ERR_SETTINGS when only
 * one of the two is NULL.  (No passage of the paper defines this call: it is
 * an interface for callers that manage device memory themselves.) */
typedef void *(*osqp_alloc_fn)(size_t bytes, void *ctx);
typedef void (*osqp_free_fn)(void *ptr, void *ctx);
osqp_int osqp_set_allocator(osqp_alloc_fn alloc, osqp_free_fn free_fn, void *ctx);

/* Number of visible HIP devices (0 when none), for callers that must gate. */
osqp_int osqp_device_count(void);

/* Properties of the current device the library sizes its launches by: compute
 * units, LDS bytes a workgroup may use, LDS bytes per CU, and the rate of the
 * device wall clock in kHz.  Any pointer may be NULL. */
osqp_int osqp_device_info(osqp_int *cu_count, osqp_int *lds_per_block, osqp_int *lds_per_cu,
                          osqp_int *wall_khz);

/* ---- single QP (Sections 3-5) ------------------------------------------ */

/* Validate and copy one QP to the device, build P's full symmetric pattern
 * and the rows of A' (= the columns of A), run the modified Ruiz
 * equilibration of Section 5.1 on the device and set the rho vector of
 * Section 5.2.  s may be NULL (defaults).  On error *out is NULL. */
osqp_int osqp_setup(osqp_solver **out, osqp_int n, osqp_int m,
                    const osqp_csr *P_upper, const osqp_float *q,
                    const osqp_csr *A, const osqp_float *l, const osqp_float *u,
                    const osqp_settings *s);

/* Run ADMM (Algorithm 1, reduced-system PCG form of Section 3.1) until a
 * status of Sections 3.3-3.4 is reached, then unscale (Section 5.1) and,
 * if enabled, polish (Section 4).  Blocks until the result is on the host.
 * The first solve starts from zero; each later one starts from the last
 * iterate and rho-bar (the warm start of Section 6, as after
 * osqp_update_vectors), unless osqp_warm_start gave another point or
 * osqp_batch_reset returned the handle to its state after setup. */
osqp_int osqp_solve(osqp_solver *h);

/* Replace q, l and/or u (NULL = unchanged), unscaled, same sizes
 * (Section 6, vectors as parameters): the stored scaling D, E, c is applied
 * and the matrices stay resident.  Rows whose l_i == u_i status changes get
 * their rho_i updated. */
osqp_int osqp_update_vectors(osqp_solver *h, const osqp_float *q,
                             const osqp_float *l, const osqp_float *u);

/* Warm start (Section 6): x0 = x, y0 = y (unscaled; NULL = keep the
 * current iterate), z0 = A x0. */
osqp_int osqp_warm_start(osqp_solver *h, const osqp_float *x, const osqp_float *y);

/* Replace the values of P and/or A with the sparsity patterns kept (Section
 * 6, matrices as parameters; the paper re-factors numerically and keeps the
 * symbolic part).  P_upper_data: the P_nnz values of the upper triangle in
 * the CSR order of the setup; A_data: the A_nnz values of A in its CSR order;
 * NULL leaves that matrix unchanged.  The new data is unscaled: the modified
 * Ruiz equilibration of Section 5.1 is recomputed on the device from it, the
 * stored factor of the reduced matrix is recomputed at the next solve, and
 * that solve is warm-started from the last solution (unscaled x, y).  P must
 * stay positive semidefinite (not checked).  Blocks until done.
 * OSQP_ERR_DIM when a count differs from the setup's, OSQP_ERR_DATA_NONFINITE
 * for NaN/inf values. */
osqp_int osqp_update_matrices(osqp_solver *h, const osqp_float *P_upper_data, osqp_int P_nnz,
                              const osqp_float *A_data, osqp_int A_nnz);

/* Copy the last solution (unscaled, FP64) to x (n) and y (m); either may be NULL. */
osqp_int osqp_get_solution(const osqp_solver *h, osqp_float *x, osqp_float *y);
osqp_int osqp_get_info(const osqp_solver *h, osqp_info *info);
void osqp_cleanup(osqp_solver *h);

/* ---- batches of independent QPs (same settings) ----------------------- */

/* Set up `count` QPs at once; they are packed block-diagonally in HBM and
 * solved together by one persistent kernel. */
osqp_int osqp_batch_setup(osqp_batch **out, osqp_int count, const osqp_problem *probs,
                          const osqp_settings *s);
/* Solve every QP of the batch (blocks until all statuses are final). */
osqp_int osqp_batch_solve(osqp_batch *b);
/* Enqueue the solve on the batch's stream without waiting (results are
 * valid after osqp_batch_sync). */
osqp_int osqp_batch_solve_async(osqp_batch *b);
/* Enqueue the solve of the `count` QPs listed in idx (distinct indices into
 * the batch, host memory, copied before return) without waiting; the other
 * QPs keep their state.  Every listed QP runs on one workgroup (the
 * whole-grid team is not used), with polishing when enabled and the QP is
 * polishable.  This is how a resident set of structures is re-solved for the
 * requests that arrived (Section 6: new vectors and warm starts, matrices and
 * factors kept).  OSQP_ERR_INDEX for an index out of range or repeated;
 * results after osqp_batch_sync. */
osqp_int osqp_batch_solve_subset_async(osqp_batch *b, const osqp_int *idx, osqp_int count);
osqp_int osqp_batch_sync(osqp_batch *b);
/* Enqueue the whole-batch solve as one replay of a HIP graph (counter reset,
 * the persistent workgroup solve, polishing), built on the first call for the
 * batch's current launch shape and rebuilt after osqp_batch_set_shape.  Same
 * results as osqp_batch_solve_async; results after osqp_batch_sync.  For
 * callers that replay the solve of resident QPs many times (Section 6:
 * parametric re-solves after update_vectors / warm_start).  Returns
 * OSQP_ERR_UNSUPPORTED when the batch holds QPs solved by the whole grid (their
 * launch is cooperative); osqp_batch_last_kernel_ms then spans the graph. */
osqp_int osqp_batch_solve_graph_async(osqp_batch *b);
/* Launch-shape tuner: switched off.  Returns OSQP_ERR_UNSUPPORTED for every
 * batch (OSQP_ERR_NOT_SETUP for a NULL handle) and leaves `out` untouched.
 * The device was lost during its GPU test in several runs without a cause
 * being shown, so no shape is timed on the device; callers apply a known
 * shape with osqp_batch_set_shape. */
osqp_int osqp_batch_autotune(osqp_batch *b, osqp_int reps, osqp_tuning *out);
/* Apply a launch shape: block_size a multiple of 64 in [64, 512] (equal to
 * settings.block_size if that is nonzero), lane_div in [1, 1024] (lanes per
 * CSR row ~ the QP's mean row length / lane_div, a power of two up to 64).
 * The grid follows the occupancy of the new workgroup size but never exceeds
 * the grid sized at setup (the per-workgroup workspaces keep their size;
 * nothing is allocated).  Waits for the batch's stream; iterates, results
 * and the scaling are kept (osqp_batch_reset redoes the scaling, whose sums
 * then run in the new shape's order, so results across shapes agree to the
 * solver's tolerance, not bitwise).  OSQP_ERR_SETTINGS for a shape out of
 * range. */
osqp_int osqp_batch_set_shape(osqp_batch *b, osqp_int block_size, osqp_int lane_div);
/* Re-run the device-side Ruiz scaling from the resident unscaled data and
 * reset every iterate to zero (a fresh solve of the same problems). */
osqp_int osqp_batch_reset(osqp_batch *b);
osqp_int osqp_batch_update_vectors(osqp_batch *b, osqp_int i, const osqp_float *q,
                                   const osqp_float *l, const osqp_float *u);
osqp_int osqp_batch_warm_start(osqp_batch *b, osqp_int i, const osqp_float *x,
                               const osqp_float *y);
/* osqp_update_matrices for problem i of a batch. */
osqp_int osqp_batch_update_matrices(osqp_batch *b, osqp_int i, const osqp_float *P_upper_data,
                                    osqp_int P_nnz, const osqp_float *A_data, osqp_int A_nnz);
/* Result of problem i: x (n_i), y (m_i) and info; any pointer may be NULL. */
osqp_int osqp_batch_get(const osqp_batch *b, osqp_int i, osqp_float *x, osqp_float *y,
                        osqp_info *info);
/* Device time in milliseconds of the last solve's main kernel (HIP events on
 * the batch's stream). */
osqp_int osqp_batch_last_kernel_ms(const osqp_batch *b, double *ms);
osqp_int osqp_batch_count(const osqp_batch *b, osqp_int *count);
/* Copy the factor of problem i's reduced matrix K = P + sigma I + A'RA
 * (scaled data, current rho; Section 3.1) to L_out as n*n row-major doubles:
 * on the dense path its Cholesky factor L (lower triangle, upper part zero);
 * on the band path G = Pi' L with L the block-bidiagonal Cholesky factor of
 * the reordered matrix Pi K Pi' (rows of L put back in variable order), so
 * that G G' = K.  Returns OSQP_ERR_NOT_SETUP when problem i uses neither
 * path or has no valid factor yet.  For checking and diagnostics. */
osqp_int osqp_batch_get_factor(const osqp_batch *b, osqp_int i, osqp_float *L_out);
void osqp_batch_cleanup(osqp_batch *b);

/* ---- continuous-batching server ----------------------------------------
 * A scheduler thread admits submitted QPs while slots (max_slots QPs on the
 * device at once), the HBM budget and a limit of launches in flight allow;
 * while the device is full, requests accumulate and are admitted together
 * when a launch drains.  Fresh QPs admitted together form a micro-batch set
 * up and solved on its own stream, so launches admitted while others run
 * overlap on the device; a fresh QP with at least 200,000 matrix entries
 * (2 nnz(A) + nnz(P) + n + m) gets a launch of its own, so that the small
 * ones admitted with it do not wait for it.  A nonzero structure_key marks QPs that share
 * matrices: first requests of new keys form a resident pool (matrices,
 * scaling, factors, iterates stay on the device) and later requests of those
 * keys are re-solved together as a subset of their pool through the vector
 * update and warm start of Section 6 (their P and A must equal the first's;
 * only q, l, u are taken).  Idle pools are evicted least recently used
 * first when the budget needs room.  Tickets are returned at submission.
 * Calls from several client threads are allowed. */
osqp_int osqp_server_create(osqp_server **out, size_t hbm_budget_bytes, osqp_int max_slots,
                            const osqp_settings *s);
/* Copy the problem and queue it.  x_ws / y_ws (may be NULL) warm start it.
 * Returns OSQP_ERR_BUDGET when the QP alone exceeds the budget, or a
 * validation code; *ticket identifies the request. */
osqp_int osqp_server_submit(osqp_server *sv, const osqp_problem *p, uint64_t structure_key,
                            const osqp_float *x_ws, const osqp_float *y_ws, uint64_t *ticket);
/* Block until request `ticket` is done; copy x (n), y (m), info and the
 * latency (completion minus submission, seconds).  Any output may be NULL.
 * Returns the request's own error code if its setup or solve failed.  A
 * ticket is collected once: OSQP_ERR_INDEX for an unknown ticket or one
 * already collected (also for a second thread waiting on the same one). */
osqp_int osqp_server_wait(osqp_server *sv, uint64_t ticket, osqp_float *x, osqp_float *y,
                          osqp_info *info, double *latency_s);
/* Counters: requests completed, micro-batches launched, peak concurrent
 * micro-batches on the device, peak HBM bytes in use.  Any pointer may be NULL. */
osqp_int osqp_server_stats(const osqp_server *sv, int64_t *completed, int64_t *batches,
                           int64_t *peak_inflight, int64_t *peak_bytes);
/* Finish every queued request, then stop the scheduler and free everything. */
void osqp_server_destroy(osqp_server *sv);

#ifdef __cplusplus
}
#endif
#endif
