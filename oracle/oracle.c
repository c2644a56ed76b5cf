/*
 * FP64 CPU oracle for the ADMM QP method (OSQP paper) -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library.  It shares nothing with the GPU path.  It follows the
 * paper's steps in order, in double precision, with a direct LDL' solve of the
 * quasi-definite KKT system (Section 3.1, direct method):
 *
 *   setup   : modified Ruiz equilibration (Section 5.1, Algorithm "Modified Ruiz
 *             equilibration"), rho vector (Section 5.2), KKT assembly (eq. kkt),
 *             minimum-degree ordering, symbolic + numeric LDL' (Section 3.1).
 *   iterate : Algorithm 1 (Section 3.2) with the z/y update written in the
 *             v-form of Section 3.3, eq. zy-update.
 *   check   : unscaled optimality and infeasibility tests (Sections 3.4, 5.1),
 *             adaptive rho-bar (Section 5.2).
 *   finish  : unscaling (Section 5.1), solution polishing with regularisation
 *             and iterative refinement (Section 4).
 *
 * Where the paper leaves a point open, the reading taken is marked "reading"
 * where it is applied.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_INF_BOUND 1e30

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void *xmalloc(size_t n) { return malloc(n ? n : 1); }
static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz ? sz : 1); }

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

void orc_default_settings(orc_settings *s) {
  /* Defaults of Section 7 (tolerances, sigma, alpha, refinement passes),
   * Section 5.2 (rho-bar^0 = 0.1) and Section 4 (delta ~ 1e-6). */
  s->rho = 0.1;
  s->sigma = 1e-6;
  s->alpha = 1.6;
  s->eps_abs = 1e-3;
  s->eps_rel = 1e-3;
  s->eps_pinf = 1e-4;
  s->eps_dinf = 1e-4;
  s->delta = 1e-6;
  s->time_limit = 0.0;
  s->max_iter = 4000;        /* reading: the paper sets no cap; 4000 here */
  s->check_every = 25;       /* reading: the paper's iteration medians are multiples of 25 */
  s->scaling_iters = 10;     /* reading: fixed number of Ruiz passes */
  s->adaptive_rho = 1;
  s->polish = 0;
  s->polish_refine_iter = 3;
}

/* ------------------------------------------------------------------------ */
/* Sparse products                                                          */
/* ------------------------------------------------------------------------ */

/* y = P x with P symmetric, stored as its upper triangle in CSR. */
static void sym_matvec(int n, const int *Pp, const int *Pi, const double *Px,
                       const double *x, double *y) {
  for (int i = 0; i < n; ++i) y[i] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int p = Pp[i]; p < Pp[i + 1]; ++p) {
      int j = Pi[p];
      y[i] += Px[p] * x[j];
      if (j != i) y[j] += Px[p] * x[i];
    }
}

/* y = A x, A m x n in CSR. */
static void csr_matvec(int m, const int *Ap, const int *Ai, const double *Ax,
                       const double *x, double *y) {
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int p = Ap[i]; p < Ap[i + 1]; ++p) s += Ax[p] * x[Ai[p]];
    y[i] = s;
  }
}

/* y = A' x, A m x n in CSR. */
static void csr_tmatvec(int m, int n, const int *Ap, const int *Ai, const double *Ax,
                        const double *x, double *y) {
  for (int j = 0; j < n; ++j) y[j] = 0.0;
  for (int i = 0; i < m; ++i)
    for (int p = Ap[i]; p < Ap[i + 1]; ++p) y[Ai[p]] += Ax[p] * x[i];
}

static double norm_inf(int n, const double *v) {
  double r = 0.0;
  for (int i = 0; i < n; ++i) r = dmax(r, fabs(v[i]));
  return r;
}

/* ------------------------------------------------------------------------ */
/* Minimum-degree ordering (Section 3.1 asks for a fill-reducing ordering;   */
/* any symmetric permutation of a quasi-definite matrix has an LDL' factor). */
/* Explicit elimination graph; nodes of very high degree are ordered last;   */
/* once the remaining graph is a clique the rest keeps its natural order.    */
/* ------------------------------------------------------------------------ */

typedef struct { int deg, node; } heap_item;

static void heap_push(heap_item *h, long *hn, heap_item it) {
  long i = (*hn)++;
  h[i] = it;
  while (i > 0) {
    long par = (i - 1) / 2;
    if (h[par].deg < h[i].deg || (h[par].deg == h[i].deg && h[par].node <= h[i].node)) break;
    heap_item t = h[par]; h[par] = h[i]; h[i] = t;
    i = par;
  }
}

static heap_item heap_pop(heap_item *h, long *hn) {
  heap_item top = h[0];
  h[0] = h[--(*hn)];
  long i = 0;
  for (;;) {
    long a = 2 * i + 1, b = a + 1, s = i;
    if (a < *hn && (h[a].deg < h[s].deg || (h[a].deg == h[s].deg && h[a].node < h[s].node))) s = a;
    if (b < *hn && (h[b].deg < h[s].deg || (h[b].deg == h[s].deg && h[b].node < h[s].node))) s = b;
    if (s == i) break;
    heap_item t = h[s]; h[s] = h[i]; h[i] = t;
    i = s;
  }
  return top;
}

int orc_mindeg(int N, const int *Kp, const int *Ki, int *perm) {
  if (N <= 0) return 0;
  int *deg0 = (int *)xcalloc((size_t)N, sizeof(int));
  for (int j = 0; j < N; ++j)
    for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
      int i = Ki[p];
      if (i != j) { deg0[i]++; deg0[j]++; }
    }
  int dthr = (int)(10.0 * sqrt((double)N));
  if (dthr < 16) dthr = 16;
  char *dense = (char *)xcalloc((size_t)N, 1);
  for (int i = 0; i < N; ++i) dense[i] = deg0[i] > dthr;

  int *len = (int *)xcalloc((size_t)N, sizeof(int));
  int *cap = (int *)xcalloc((size_t)N, sizeof(int));
  int **adj = (int **)xcalloc((size_t)N, sizeof(int *));
  for (int i = 0; i < N; ++i) {
    cap[i] = dense[i] ? 1 : (deg0[i] > 0 ? deg0[i] : 1);
    adj[i] = (int *)xmalloc(sizeof(int) * (size_t)cap[i]);
  }
  for (int j = 0; j < N; ++j)
    for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
      int i = Ki[p];
      if (i == j || dense[i] || dense[j]) continue;
      adj[i][len[i]++] = j;
      adj[j][len[j]++] = i;
    }
  /* remove duplicate edges (a pattern may list an entry twice) */
  long *mark = (long *)xcalloc((size_t)N, sizeof(long));
  long stamp = 0;
  for (int i = 0; i < N; ++i) {
    ++stamp;
    int w = 0;
    for (int t = 0; t < len[i]; ++t) {
      int k = adj[i][t];
      if (mark[k] != stamp) { mark[k] = stamp; adj[i][w++] = k; }
    }
    len[i] = w;
  }

  char *done = (char *)xcalloc((size_t)N, 1);
  long hcap = 4L * N + 16, hn = 0;
  heap_item *heap = (heap_item *)xmalloc(sizeof(heap_item) * (size_t)hcap);
  int remaining = 0;
  for (int i = 0; i < N; ++i)
    if (!dense[i]) { heap_item it = {len[i], i}; heap_push(heap, &hn, it); remaining++; }

  int *nb = (int *)xmalloc(sizeof(int) * (size_t)N);
  int k = 0;
  while (remaining > 0) {
    heap_item it = heap_pop(heap, &hn);
    int v = it.node;
    if (done[v] || it.deg != len[v]) continue;
    if (len[v] == remaining - 1) {
      /* the remaining graph is complete: keep the natural order */
      for (int i = 0; i < N; ++i)
        if (!dense[i] && !done[i]) { perm[k++] = i; done[i] = 1; }
      remaining = 0;
      break;
    }
    perm[k++] = v;
    done[v] = 1;
    remaining--;
    int nv = len[v];
    memcpy(nb, adj[v], sizeof(int) * (size_t)nv);
    for (int a = 0; a < nv; ++a) {
      int u = nb[a];
      ++stamp;
      int w = 0;
      for (int t = 0; t < len[u]; ++t) {
        int x = adj[u][t];
        if (x == v) continue;
        mark[x] = stamp;
        adj[u][w++] = x;
      }
      len[u] = w;
      for (int b = 0; b < nv; ++b) {
        int x = nb[b];
        if (x == u || mark[x] == stamp) continue;
        if (len[u] == cap[u]) {
          cap[u] = 2 * cap[u] + 4;
          adj[u] = (int *)realloc(adj[u], sizeof(int) * (size_t)cap[u]);
        }
        adj[u][len[u]++] = x;
        mark[x] = stamp;
      }
      if (hn + 1 >= hcap) {
        hcap *= 2;
        heap = (heap_item *)realloc(heap, sizeof(heap_item) * (size_t)hcap);
      }
      heap_item ni = {len[u], u};
      heap_push(heap, &hn, ni);
    }
    free(adj[v]); adj[v] = NULL; len[v] = 0;
  }
  for (int i = 0; i < N; ++i)
    if (dense[i]) perm[k++] = i;

  for (int i = 0; i < N; ++i) free(adj[i]);
  free(adj); free(len); free(cap); free(deg0); free(dense); free(mark);
  free(done); free(heap); free(nb);
  return k == N ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Sparse LDL' (Section 3.1): elimination tree + symbolic counts, then the   */
/* up-looking numeric factorisation; D^-1 is stored so solves do not divide. */
/* The method is the published up-looking sparse LDL' of T. Davis (2005),    */
/* the basis Section 7 names for the paper's own direct solver, written out  */
/* here from its description.                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int N;
  int *perm, *pinv;          /* perm[k] = original index of pivot k */
  int *Cp, *Ci; double *Cx;  /* permuted upper triangle, CSC */
  int *map;                  /* position in Cx of each original upper entry */
  int *parent, *Lnz, *Lp, *Li;
  double *Lx, *D, *Dinv;
} ldl_t;

static void ldl_free(ldl_t *f) {
  if (!f) return;
  free(f->perm); free(f->pinv); free(f->Cp); free(f->Ci); free(f->Cx); free(f->map);
  free(f->parent); free(f->Lnz); free(f->Lp); free(f->Li); free(f->Lx); free(f->D);
  free(f->Dinv);
  memset(f, 0, sizeof(*f));
}

/* Ordering + permuted pattern + symbolic factorisation. */
static int ldl_symbolic(ldl_t *f, int N, const int *Kp, const int *Ki) {
  memset(f, 0, sizeof(*f));
  f->N = N;
  f->perm = (int *)xmalloc(sizeof(int) * (size_t)N);
  f->pinv = (int *)xmalloc(sizeof(int) * (size_t)N);
  if (orc_mindeg(N, Kp, Ki, f->perm) != 0) return -1;
  for (int k = 0; k < N; ++k) f->pinv[f->perm[k]] = k;
  int nnz = Kp[N];
  f->Cp = (int *)xcalloc((size_t)N + 1, sizeof(int));
  f->Ci = (int *)xmalloc(sizeof(int) * (size_t)nnz);
  f->Cx = (double *)xcalloc((size_t)nnz, sizeof(double));
  f->map = (int *)xmalloc(sizeof(int) * (size_t)nnz);
  for (int j = 0; j < N; ++j)
    for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
      int a = f->pinv[Ki[p]], b = f->pinv[j];
      f->Cp[(a > b ? a : b) + 1]++;
    }
  for (int j = 0; j < N; ++j) f->Cp[j + 1] += f->Cp[j];
  int *next = (int *)xmalloc(sizeof(int) * (size_t)N);
  memcpy(next, f->Cp, sizeof(int) * (size_t)N);
  for (int j = 0; j < N; ++j)
    for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
      int a = f->pinv[Ki[p]], b = f->pinv[j];
      int col = a > b ? a : b, row = a > b ? b : a;
      int q = next[col]++;
      f->Ci[q] = row;
      f->map[p] = q;
    }
  free(next);
  /* elimination tree and column counts of L */
  f->parent = (int *)xmalloc(sizeof(int) * (size_t)N);
  f->Lnz = (int *)xcalloc((size_t)N, sizeof(int));
  int *flag = (int *)xmalloc(sizeof(int) * (size_t)N);
  for (int k = 0; k < N; ++k) {
    f->parent[k] = -1;
    flag[k] = k;
    for (int p = f->Cp[k]; p < f->Cp[k + 1]; ++p) {
      int i = f->Ci[p];
      if (i >= k) continue;
      for (; flag[i] != k; i = f->parent[i]) {
        if (f->parent[i] == -1) f->parent[i] = k;
        f->Lnz[i]++;
        flag[i] = k;
      }
    }
  }
  free(flag);
  f->Lp = (int *)xmalloc(sizeof(int) * ((size_t)N + 1));
  f->Lp[0] = 0;
  for (int k = 0; k < N; ++k) f->Lp[k + 1] = f->Lp[k] + f->Lnz[k];
  f->Li = (int *)xmalloc(sizeof(int) * (size_t)f->Lp[N]);
  f->Lx = (double *)xmalloc(sizeof(double) * (size_t)f->Lp[N]);
  f->D = (double *)xmalloc(sizeof(double) * (size_t)N);
  f->Dinv = (double *)xmalloc(sizeof(double) * (size_t)N);
  return 0;
}

/* Numeric factorisation of the matrix whose upper-CSC values are Kx
 * (same pattern as given to ldl_symbolic). */
static int ldl_numeric(ldl_t *f, const int *Kp, const double *Kx) {
  int N = f->N;
  for (int p = 0; p < f->Cp[N]; ++p) f->Cx[p] = 0.0;
  for (int p = 0; p < Kp[N]; ++p) f->Cx[f->map[p]] += Kx[p];
  double *Y = (double *)xcalloc((size_t)N, sizeof(double));
  int *pattern = (int *)xmalloc(sizeof(int) * (size_t)N);
  int *flag = (int *)xmalloc(sizeof(int) * (size_t)N);
  int rc = 0;
  for (int k = 0; k < N; ++k) f->Lnz[k] = 0;
  for (int k = 0; k < N; ++k) {
    /* pattern of row k of L = reach of column k's entries in the etree */
    int top = N;
    flag[k] = k;
    Y[k] = 0.0;
    for (int p = f->Cp[k]; p < f->Cp[k + 1]; ++p) {
      int i = f->Ci[p];
      Y[i] += f->Cx[p];
      int len = 0;
      for (; flag[i] != k; i = f->parent[i]) {
        pattern[len++] = i;
        flag[i] = k;
      }
      while (len > 0) pattern[--top] = pattern[--len];
    }
    f->D[k] = Y[k];
    Y[k] = 0.0;
    for (; top < N; ++top) {
      int i = pattern[top];
      double yi = Y[i];
      Y[i] = 0.0;
      int p2 = f->Lp[i] + f->Lnz[i];
      for (int p = f->Lp[i]; p < p2; ++p) Y[f->Li[p]] -= f->Lx[p] * yi;
      double lki = yi / f->D[i];
      f->D[k] -= lki * yi;
      f->Li[p2] = k;
      f->Lx[p2] = lki;
      f->Lnz[i]++;
    }
    if (f->D[k] == 0.0 || !isfinite(f->D[k])) { rc = -2; break; }
    f->Dinv[k] = 1.0 / f->D[k];
  }
  free(Y); free(pattern); free(flag);
  return rc;
}

/* Solve K x = b with the factors (forward, diagonal, backward). */
static void ldl_solve(const ldl_t *f, const double *b, double *x, double *work) {
  int N = f->N;
  for (int k = 0; k < N; ++k) work[k] = b[f->perm[k]];
  for (int j = 0; j < N; ++j) {
    double wj = work[j];
    for (int p = f->Lp[j]; p < f->Lp[j] + f->Lnz[j]; ++p) work[f->Li[p]] -= f->Lx[p] * wj;
  }
  for (int j = 0; j < N; ++j) work[j] *= f->Dinv[j];
  for (int j = N - 1; j >= 0; --j) {
    double s = work[j];
    for (int p = f->Lp[j]; p < f->Lp[j] + f->Lnz[j]; ++p) s -= f->Lx[p] * work[f->Li[p]];
    work[j] = s;
  }
  for (int k = 0; k < N; ++k) x[f->perm[k]] = work[k];
}

int orc_ldl_solve(int N, const int *Kp, const int *Ki, const double *Kx,
                  const double *b, double *x) {
  ldl_t f;
  int rc = ldl_symbolic(&f, N, Kp, Ki);
  if (rc == 0) rc = ldl_numeric(&f, Kp, Kx);
  if (rc == 0) {
    double *w = (double *)xmalloc(sizeof(double) * (size_t)N);
    ldl_solve(&f, b, x, w);
    free(w);
  }
  ldl_free(&f);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Working copy of the (scaled) problem                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n, m;
  int *Pp, *Pi; double *Px;   /* upper CSR (copy, scaled in place) */
  int *Ap, *Ai; double *Ax;   /* CSR (copy, scaled in place) */
  double *q, *l, *u;
  double *D, *E, c;           /* scaling: xbar = D^-1 x, ybar = c E^-1 y */
  double *Dinv, *Einv;
} work_qp;

static void wq_free(work_qp *w) {
  free(w->Pp); free(w->Pi); free(w->Px); free(w->Ap); free(w->Ai); free(w->Ax);
  free(w->q); free(w->l); free(w->u); free(w->D); free(w->E); free(w->Dinv); free(w->Einv);
}

static void wq_copy(work_qp *w, const orc_problem *pb) {
  int n = pb->n, m = pb->m;
  w->n = n; w->m = m;
  int pn = pb->P_indptr[n], an = pb->A_indptr[m];
  w->Pp = (int *)xmalloc(sizeof(int) * ((size_t)n + 1));
  w->Pi = (int *)xmalloc(sizeof(int) * (size_t)pn);
  w->Px = (double *)xmalloc(sizeof(double) * (size_t)pn);
  memcpy(w->Pp, pb->P_indptr, sizeof(int) * ((size_t)n + 1));
  memcpy(w->Pi, pb->P_indices, sizeof(int) * (size_t)pn);
  memcpy(w->Px, pb->P_data, sizeof(double) * (size_t)pn);
  w->Ap = (int *)xmalloc(sizeof(int) * ((size_t)m + 1));
  w->Ai = (int *)xmalloc(sizeof(int) * (size_t)an);
  w->Ax = (double *)xmalloc(sizeof(double) * (size_t)an);
  memcpy(w->Ap, pb->A_indptr, sizeof(int) * ((size_t)m + 1));
  memcpy(w->Ai, pb->A_indices, sizeof(int) * (size_t)an);
  memcpy(w->Ax, pb->A_data, sizeof(double) * (size_t)an);
  w->q = (double *)xmalloc(sizeof(double) * (size_t)n);
  memcpy(w->q, pb->q, sizeof(double) * (size_t)n);
  w->l = (double *)xmalloc(sizeof(double) * (size_t)m);
  w->u = (double *)xmalloc(sizeof(double) * (size_t)m);
  for (int i = 0; i < m; ++i) {
    /* reading: |b| >= 1e30 is an infinite bound */
    w->l[i] = pb->l[i] <= -ORC_INF_BOUND ? -INFINITY : pb->l[i];
    w->u[i] = pb->u[i] >= ORC_INF_BOUND ? INFINITY : pb->u[i];
  }
  w->D = (double *)xmalloc(sizeof(double) * (size_t)n);
  w->E = (double *)xmalloc(sizeof(double) * (size_t)m);
  w->Dinv = (double *)xmalloc(sizeof(double) * (size_t)n);
  w->Einv = (double *)xmalloc(sizeof(double) * (size_t)m);
  for (int j = 0; j < n; ++j) w->D[j] = 1.0;
  for (int i = 0; i < m; ++i) w->E[i] = 1.0;
  w->c = 1.0;
}

/* Modified Ruiz equilibration (Section 5.1, Algorithm "Modified Ruiz
 * equilibration"), a fixed number of passes (reading). */
static void ruiz(work_qp *w, int iters) {
  int n = w->n, m = w->m;
  double *dx = (double *)xmalloc(sizeof(double) * (size_t)n);
  double *dz = (double *)xmalloc(sizeof(double) * (size_t)m);
  double *coln = (double *)xmalloc(sizeof(double) * (size_t)n);
  for (int it = 0; it < iters; ++it) {
    /* infinity norm of every column of M = [P A'; A 0] */
    for (int j = 0; j < n; ++j) dx[j] = 0.0;
    for (int i = 0; i < m; ++i) dz[i] = 0.0;
    for (int i = 0; i < n; ++i)
      for (int p = w->Pp[i]; p < w->Pp[i + 1]; ++p) {
        double a = fabs(w->Px[p]);
        int j = w->Pi[p];
        dx[j] = dmax(dx[j], a);
        dx[i] = dmax(dx[i], a);
      }
    for (int i = 0; i < m; ++i)
      for (int p = w->Ap[i]; p < w->Ap[i + 1]; ++p) {
        double a = fabs(w->Ax[p]);
        int j = w->Ai[p];
        dx[j] = dmax(dx[j], a);
        dz[i] = dmax(dz[i], a);
      }
    /* delta_i = 1/sqrt(norm); reading: norms below 1e-4 count as 1,
     * norms above 1e4 are clamped to 1e4 */
    for (int j = 0; j < n; ++j) {
      double v = dx[j] < 1e-4 ? 1.0 : dmin(dx[j], 1e4);
      dx[j] = 1.0 / sqrt(v);
    }
    for (int i = 0; i < m; ++i) {
      double v = dz[i] < 1e-4 ? 1.0 : dmin(dz[i], 1e4);
      dz[i] = 1.0 / sqrt(v);
    }
    /* scale P, q, A, l, u */
    for (int i = 0; i < n; ++i)
      for (int p = w->Pp[i]; p < w->Pp[i + 1]; ++p) w->Px[p] *= dx[i] * dx[w->Pi[p]];
    for (int j = 0; j < n; ++j) w->q[j] *= dx[j];
    for (int i = 0; i < m; ++i) {
      for (int p = w->Ap[i]; p < w->Ap[i + 1]; ++p) w->Ax[p] *= dz[i] * dx[w->Ai[p]];
      w->l[i] *= dz[i];
      w->u[i] *= dz[i];
    }
    for (int j = 0; j < n; ++j) w->D[j] *= dx[j];
    for (int i = 0; i < m; ++i) w->E[i] *= dz[i];
    /* cost scaling: gamma = 1 / max(mean_j ||Pbar_j||_inf, ||qbar||_inf) */
    for (int j = 0; j < n; ++j) coln[j] = 0.0;
    for (int i = 0; i < n; ++i)
      for (int p = w->Pp[i]; p < w->Pp[i + 1]; ++p) {
        double a = fabs(w->Px[p]);
        int j = w->Pi[p];
        coln[j] = dmax(coln[j], a);
        coln[i] = dmax(coln[i], a);
      }
    double mean = 0.0;
    for (int j = 0; j < n; ++j) mean += coln[j];
    mean /= (double)n;
    double s = dmax(mean, norm_inf(n, w->q));
    /* reading: gamma = 1 if P and q vanish; else clamped to [1e-4, 1e4] */
    double gamma = s == 0.0 ? 1.0 : dmin(dmax(1.0 / s, 1e-4), 1e4);
    for (int p = 0; p < w->Pp[n]; ++p) w->Px[p] *= gamma;
    for (int j = 0; j < n; ++j) w->q[j] *= gamma;
    w->c *= gamma;
  }
  for (int j = 0; j < n; ++j) w->Dinv[j] = 1.0 / w->D[j];
  for (int i = 0; i < m; ++i) w->Einv[i] = 1.0 / w->E[i];
  free(dx); free(dz); free(coln);
}

int orc_ruiz(const orc_problem *pb, int iters, double *D, double *E, double *c) {
  work_qp w;
  wq_copy(&w, pb);
  ruiz(&w, iters);
  memcpy(D, w.D, sizeof(double) * (size_t)pb->n);
  memcpy(E, w.E, sizeof(double) * (size_t)pb->m);
  *c = w.c;
  wq_free(&w);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* KKT matrix of eq. kkt, upper triangle in CSC:                             */
/*   [ P + sigma I   A'        ]                                             */
/*   [ A             -diag(1/rho) ]                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  int N;
  int *Kp, *Ki; double *Kx;
  int *diag_pos;   /* position of each diagonal entry */
} kkt_t;

static void kkt_free(kkt_t *k) { free(k->Kp); free(k->Ki); free(k->Kx); free(k->diag_pos); }

/* rows: the constraint rows to include (all rows for the ADMM system, the
 * active rows for polishing); diag_x added to P's diagonal, diag_c[r] is the
 * (2,2)-block diagonal for included row r. */
static void kkt_build(kkt_t *K, const work_qp *w, int nrows, const int *rows,
                      double diag_x, const double *diag_c) {
  int n = w->n;
  int N = n + nrows;
  K->N = N;
  /* column counts: P upper CSR row i = entries (i, j>=i) -> column j of upper CSC */
  int *cnt = (int *)xcalloc((size_t)N + 1, sizeof(int));
  for (int i = 0; i < n; ++i)
    for (int p = w->Pp[i]; p < w->Pp[i + 1]; ++p)
      if (w->Pi[p] != i) cnt[w->Pi[p]]++;
  for (int j = 0; j < n; ++j) cnt[j]++;   /* one diagonal slot per column */
  for (int r = 0; r < nrows; ++r) {
    int i = rows[r];
    cnt[n + r] = (w->Ap[i + 1] - w->Ap[i]) + 1;
  }
  K->Kp = (int *)xmalloc(sizeof(int) * ((size_t)N + 1));
  K->Kp[0] = 0;
  for (int j = 0; j < N; ++j) K->Kp[j + 1] = K->Kp[j] + cnt[j];
  int nnz = K->Kp[N];
  K->Ki = (int *)xmalloc(sizeof(int) * (size_t)nnz);
  K->Kx = (double *)xcalloc((size_t)nnz, sizeof(double));
  K->diag_pos = (int *)xmalloc(sizeof(int) * (size_t)N);
  int *next = cnt;
  for (int j = 0; j < N; ++j) next[j] = K->Kp[j];
  for (int i = 0; i < n; ++i)
    for (int p = w->Pp[i]; p < w->Pp[i + 1]; ++p) {
      int j = w->Pi[p];
      if (j == i) continue;
      int q = next[j]++;
      K->Ki[q] = i;
      K->Kx[q] = w->Px[p];
    }
  for (int j = 0; j < n; ++j) {
    int q = next[j]++;
    K->Ki[q] = j;
    K->Kx[q] = diag_x;
    K->diag_pos[j] = q;
  }
  for (int i = 0; i < n; ++i)
    for (int p = w->Pp[i]; p < w->Pp[i + 1]; ++p)
      if (w->Pi[p] == i) K->Kx[K->diag_pos[i]] += w->Px[p];
  for (int r = 0; r < nrows; ++r) {
    int i = rows[r];
    for (int p = w->Ap[i]; p < w->Ap[i + 1]; ++p) {
      int q = next[n + r]++;
      K->Ki[q] = w->Ai[p];
      K->Kx[q] = w->Ax[p];
    }
    int q = next[n + r]++;
    K->Ki[q] = n + r;
    K->Kx[q] = diag_c[r];
    K->diag_pos[n + r] = q;
  }
  free(cnt);
}

/* ------------------------------------------------------------------------ */
/* Termination checks (Sections 3.4 and 5.1, unscaled criteria)              */
/* ------------------------------------------------------------------------ */

typedef struct {
  double prim_res, dual_res, eps_prim, eps_dual;
  double prim_res_s, dual_res_s, prim_norm_s, dual_norm_s;   /* scaled, for rho-bar */
} resid_t;

/* residuals of the scaled iterate (xb, zb, yb), reported unscaled */
static void residuals(const work_qp *w, const orc_settings *s, const double *xb,
                      const double *zb, const double *yb, double *Ax, double *Px,
                      double *Aty, resid_t *r) {
  int n = w->n, m = w->m;
  csr_matvec(m, w->Ap, w->Ai, w->Ax, xb, Ax);
  sym_matvec(n, w->Pp, w->Pi, w->Px, xb, Px);
  csr_tmatvec(m, n, w->Ap, w->Ai, w->Ax, yb, Aty);
  double pr = 0, ax = 0, zz = 0, prs = 0, axs = 0, zzs = 0;
  for (int i = 0; i < m; ++i) {
    double e = w->Einv[i];
    pr = dmax(pr, fabs(e * (Ax[i] - zb[i])));
    ax = dmax(ax, fabs(e * Ax[i]));
    zz = dmax(zz, fabs(e * zb[i]));
    prs = dmax(prs, fabs(Ax[i] - zb[i]));
    axs = dmax(axs, fabs(Ax[i]));
    zzs = dmax(zzs, fabs(zb[i]));
  }
  double dr = 0, px = 0, aty = 0, qq = 0, drs = 0, pxs = 0, atys = 0, qqs = 0;
  for (int j = 0; j < n; ++j) {
    double d = w->Dinv[j];
    double rd = Px[j] + w->q[j] + Aty[j];
    dr = dmax(dr, fabs(d * rd));
    px = dmax(px, fabs(d * Px[j]));
    aty = dmax(aty, fabs(d * Aty[j]));
    qq = dmax(qq, fabs(d * w->q[j]));
    drs = dmax(drs, fabs(rd));
    pxs = dmax(pxs, fabs(Px[j]));
    atys = dmax(atys, fabs(Aty[j]));
    qqs = dmax(qqs, fabs(w->q[j]));
  }
  double cinv = 1.0 / w->c;
  r->prim_res = pr;
  r->eps_prim = s->eps_abs + s->eps_rel * dmax(ax, zz);
  r->dual_res = cinv * dr;
  r->eps_dual = s->eps_abs + s->eps_rel * cinv * dmax(px, dmax(aty, qq));
  r->prim_res_s = prs;
  r->prim_norm_s = dmax(axs, zzs);
  r->dual_res_s = drs;
  r->dual_norm_s = dmax(pxs, dmax(atys, qqs));
}

/* Primal infeasibility test on dy (Section 5.1).  Readings: the certificate
 * needs ||E dy|| > 0; the support-function term must be strictly below
 * -eps * ||E dy||; only rows with dy_i > 0 use u_i and only rows with
 * dy_i < 0 use l_i; an infinite bound met with a nonzero dy of its sign
 * fails the test. */
static int primal_infeasible(const work_qp *w, const orc_settings *s, const double *dy,
                             double *tmp_n) {
  int n = w->n, m = w->m;
  double ndy = 0.0;
  for (int i = 0; i < m; ++i) ndy = dmax(ndy, fabs(w->E[i] * dy[i]));
  if (!(ndy > 0.0)) return 0;
  double supp = 0.0;
  for (int i = 0; i < m; ++i) {
    if (dy[i] > 0.0) {
      if (isinf(w->u[i])) return 0;
      supp += w->u[i] * dy[i];
    } else if (dy[i] < 0.0) {
      if (isinf(w->l[i])) return 0;
      supp += w->l[i] * dy[i];
    }
  }
  if (!(supp < -s->eps_pinf * ndy)) return 0;
  csr_tmatvec(m, n, w->Ap, w->Ai, w->Ax, dy, tmp_n);
  double nat = 0.0;
  for (int j = 0; j < n; ++j) nat = dmax(nat, fabs(w->Dinv[j] * tmp_n[j]));
  return nat <= s->eps_pinf * ndy;
}

/* Dual infeasibility test on dx (Section 5.1).  Readings: ||D dx|| > 0;
 * q'dx strictly below -c eps ||D dx||; rows with both bounds infinite
 * carry no condition. */
static int dual_infeasible(const work_qp *w, const orc_settings *s, const double *dx,
                           double *tmp_n, double *tmp_m) {
  int n = w->n, m = w->m;
  double ndx = 0.0;
  for (int j = 0; j < n; ++j) ndx = dmax(ndx, fabs(w->D[j] * dx[j]));
  if (!(ndx > 0.0)) return 0;
  double qdx = 0.0;
  for (int j = 0; j < n; ++j) qdx += w->q[j] * dx[j];
  double tol = s->eps_dinf * ndx;
  if (!(qdx < -w->c * tol)) return 0;
  sym_matvec(n, w->Pp, w->Pi, w->Px, dx, tmp_n);
  double npdx = 0.0;
  for (int j = 0; j < n; ++j) npdx = dmax(npdx, fabs(w->Dinv[j] * tmp_n[j]));
  if (!(npdx <= w->c * tol)) return 0;
  csr_matvec(m, w->Ap, w->Ai, w->Ax, dx, tmp_m);
  for (int i = 0; i < m; ++i) {
    double v = w->Einv[i] * tmp_m[i];
    int lf = !isinf(w->l[i]), uf = !isinf(w->u[i]);
    if (lf && uf) {
      if (fabs(v) > tol) return 0;
    } else if (lf && !uf) {
      if (v < -tol) return 0;
    } else if (!lf && uf) {
      if (v > tol) return 0;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Polishing (Section 4): active sets from y, regularised reduced KKT         */
/* (eq. kkt_polish_reg), fixed iterative-refinement passes (eq.              */
/* iterative_refinement) against the unregularised matrix (eq. kkt_polish).  */
/* ------------------------------------------------------------------------ */

static int polish(const work_qp *w, const orc_settings *s, double *xb, double *zb,
                  double *yb, resid_t *res, const resid_t *admm_res) {
  int n = w->n, m = w->m;
  int *rows = (int *)xmalloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
  int na = 0;
  for (int i = 0; i < m; ++i)
    if (yb[i] < 0.0 || yb[i] > 0.0) rows[na++] = i;
  int N = n + na;
  double *dc = (double *)xmalloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
  for (int r = 0; r < na; ++r) dc[r] = -s->delta;
  kkt_t K;
  kkt_build(&K, w, na, rows, s->delta, dc);
  ldl_t f;
  int rc = ldl_symbolic(&f, N, K.Kp, K.Ki);
  if (rc == 0) rc = ldl_numeric(&f, K.Kp, K.Kx);
  int accepted = -1;
  if (rc == 0) {
    double *g = (double *)xmalloc(sizeof(double) * (size_t)N);
    double *t = (double *)xmalloc(sizeof(double) * (size_t)N);
    double *r = (double *)xmalloc(sizeof(double) * (size_t)N);
    double *dt = (double *)xmalloc(sizeof(double) * (size_t)N);
    double *wk = (double *)xmalloc(sizeof(double) * (size_t)N);
    for (int j = 0; j < n; ++j) g[j] = -w->q[j];
    for (int a = 0; a < na; ++a) {
      int i = rows[a];
      g[n + a] = yb[i] < 0.0 ? w->l[i] : w->u[i];
    }
    ldl_solve(&f, g, t, wk);
    /* iterative refinement: t += (K + dK)^-1 (g - K t), K without delta */
    for (int it = 0; it < s->polish_refine_iter; ++it) {
      sym_matvec(n, w->Pp, w->Pi, w->Px, t, r);
      for (int a = 0; a < na; ++a) {
        int i = rows[a];
        double sa = 0.0;
        for (int p = w->Ap[i]; p < w->Ap[i + 1]; ++p) {
          sa += w->Ax[p] * t[w->Ai[p]];
          r[w->Ai[p]] += w->Ax[p] * t[n + a];
        }
        r[n + a] = sa;
      }
      for (int k = 0; k < N; ++k) r[k] = g[k] - r[k];
      ldl_solve(&f, r, dt, wk);
      for (int k = 0; k < N; ++k) t[k] += dt[k];
    }
    double *xp = (double *)xmalloc(sizeof(double) * (size_t)n);
    double *yp = (double *)xcalloc((size_t)(m > 0 ? m : 1), sizeof(double));
    double *zp = (double *)xmalloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *Ax = (double *)xmalloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *Px = (double *)xmalloc(sizeof(double) * (size_t)n);
    double *Aty = (double *)xmalloc(sizeof(double) * (size_t)n);
    memcpy(xp, t, sizeof(double) * (size_t)n);
    for (int a = 0; a < na; ++a) yp[rows[a]] = t[n + a];
    /* z = projection of A x onto [l, u] */
    csr_matvec(m, w->Ap, w->Ai, w->Ax, xp, zp);
    for (int i = 0; i < m; ++i) zp[i] = dmin(dmax(zp[i], w->l[i]), w->u[i]);
    resid_t pr;
    residuals(w, s, xp, zp, yp, Ax, Px, Aty, &pr);
    /* reading: accept when both residuals do not exceed the ADMM ones and
     * the duals of the active inequality rows keep their signs.  Section 4
     * accepts a point that meets the optimality conditions; on a row with
     * l_i = u_i both bounds are active, so its dual may take either sign and
     * is not tested (l and u are scaled by the same E_i, so the equality
     * holds here exactly when it holds on the input) */
    int ok = isfinite(pr.prim_res) && isfinite(pr.dual_res) &&
             pr.prim_res <= admm_res->prim_res && pr.dual_res <= admm_res->dual_res;
    for (int a = 0; a < na && ok; ++a) {
      int i = rows[a];
      if (w->l[i] == w->u[i]) continue;
      if (yb[i] < 0.0 && yp[i] > 0.0) ok = 0;
      if (yb[i] > 0.0 && yp[i] < 0.0) ok = 0;
    }
    if (ok) {
      memcpy(xb, xp, sizeof(double) * (size_t)n);
      memcpy(yb, yp, sizeof(double) * (size_t)m);
      memcpy(zb, zp, sizeof(double) * (size_t)m);
      *res = pr;
      accepted = 1;
    }
    free(g); free(t); free(r); free(dt); free(wk);
    free(xp); free(yp); free(zp); free(Ax); free(Px); free(Aty);
  }
  ldl_free(&f);
  kkt_free(&K);
  free(rows); free(dc);
  return accepted;
}

/* ------------------------------------------------------------------------ */
/* The solver                                                                */
/* ------------------------------------------------------------------------ */

static void set_rho(const work_qp *w, const double *l_in, const double *u_in, double rho_bar,
                    double *rho, double *rhoinv) {
  /* Section 5.2: rho_i = rho-bar for l_i != u_i and 1e3 rho-bar for l_i == u_i
   * (reading: the equality test is exact, on the unscaled input) */
  for (int i = 0; i < w->m; ++i) {
    rho[i] = (l_in[i] == u_in[i]) ? 1e3 * rho_bar : rho_bar;
    rhoinv[i] = 1.0 / rho[i];
  }
}

/* Section 5.2 rule for rho-bar: the square root of the ratio of the scaled
 * primal residual, normalised by max(||Abar xbar||, ||zbar||), to the scaled
 * dual residual, normalised by max(||Pbar xbar||, ||Abar' ybar||, ||qbar||),
 * multiplies the current value.  Readings: no update when a normaliser or
 * the dual residual is zero; the new value is clamped to [1e-6, 1e6]; it is
 * taken when it is at least 5 times larger or smaller than the current one
 * (the paper's time-based condition is replaced by evaluating the rule at
 * every termination check).  Returns the value to use: the new one, or
 * rho_bar itself when the rule does not apply. */
double orc_rho_update(double rho_bar, double prim_res, double prim_norm, double dual_res,
                      double dual_norm) {
  if (!(prim_norm > 0.0) || !(dual_norm > 0.0) || !(dual_res > 0.0)) return rho_bar;
  double ratio = (prim_res / prim_norm) / (dual_res / dual_norm);
  double rnew = rho_bar * sqrt(ratio);
  rnew = dmin(dmax(rnew, 1e-6), 1e6);
  if (rnew >= 5.0 * rho_bar || rnew <= rho_bar / 5.0) return rnew;
  return rho_bar;
}

int orc_solve(const orc_problem *pb, const orc_settings *s, const double *x_ws,
              const double *y_ws, double *x_out, double *y_out, double *z_out,
              orc_info *info) {
  double t0 = now_s();
  memset(info, 0, sizeof(*info));
  int n = pb->n, m = pb->m;
  work_qp w;
  wq_copy(&w, pb);
  ruiz(&w, s->scaling_iters);

  double rho_bar = s->rho;
  double *rho = (double *)xmalloc(sizeof(double) * (size_t)(m ? m : 1));
  double *rhoinv = (double *)xmalloc(sizeof(double) * (size_t)(m ? m : 1));
  set_rho(&w, pb->l, pb->u, rho_bar, rho, rhoinv);

  int *allrows = (int *)xmalloc(sizeof(int) * (size_t)(m ? m : 1));
  for (int i = 0; i < m; ++i) allrows[i] = i;
  double *dc = (double *)xmalloc(sizeof(double) * (size_t)(m ? m : 1));
  for (int i = 0; i < m; ++i) dc[i] = -rhoinv[i];
  kkt_t K;
  kkt_build(&K, &w, m, allrows, s->sigma, dc);
  int N = n + m;
  ldl_t f;
  int rc = ldl_symbolic(&f, N, K.Kp, K.Ki);
  if (rc == 0) rc = ldl_numeric(&f, K.Kp, K.Kx);
  if (rc != 0) {
    ldl_free(&f); kkt_free(&K); wq_free(&w);
    free(rho); free(rhoinv); free(allrows); free(dc);
    return rc;
  }
  double t1 = now_s();
  info->setup_time = t1 - t0;

  double *xb = (double *)xcalloc((size_t)n, sizeof(double));
  double *zb = (double *)xcalloc((size_t)(m ? m : 1), sizeof(double));
  double *yb = (double *)xcalloc((size_t)(m ? m : 1), sizeof(double));
  double *xprev = (double *)xmalloc(sizeof(double) * (size_t)n);
  double *yprev = (double *)xmalloc(sizeof(double) * (size_t)(m ? m : 1));
  double *rhs = (double *)xmalloc(sizeof(double) * (size_t)N);
  double *sol = (double *)xmalloc(sizeof(double) * (size_t)N);
  double *wk = (double *)xmalloc(sizeof(double) * (size_t)N);
  double *Ax = (double *)xmalloc(sizeof(double) * (size_t)(m ? m : 1));
  double *Px = (double *)xmalloc(sizeof(double) * (size_t)n);
  double *Aty = (double *)xmalloc(sizeof(double) * (size_t)n);
  double *dx = (double *)xmalloc(sizeof(double) * (size_t)n);
  double *dy = (double *)xmalloc(sizeof(double) * (size_t)(m ? m : 1));

  /* initial iterate: zeros (reading), or the warm start of Section 6:
   * xbar = D^-1 x, ybar = c E^-1 y, zbar = Abar xbar */
  if (x_ws) {
    for (int j = 0; j < n; ++j) xb[j] = w.Dinv[j] * x_ws[j];
    csr_matvec(m, w.Ap, w.Ai, w.Ax, xb, zb);
  }
  if (y_ws)
    for (int i = 0; i < m; ++i) yb[i] = w.c * w.Einv[i] * y_ws[i];

  int status = ORC_UNSOLVED;
  resid_t res;
  memset(&res, 0, sizeof(res));
  int k = 0;
  const double alpha = s->alpha, sigma = s->sigma;
  while (k < s->max_iter) {
    memcpy(xprev, xb, sizeof(double) * (size_t)n);
    memcpy(yprev, yb, sizeof(double) * (size_t)m);
    /* Algorithm 1, linear system (eq. kkt) */
    for (int j = 0; j < n; ++j) rhs[j] = sigma * xb[j] - w.q[j];
    for (int i = 0; i < m; ++i) rhs[n + i] = zb[i] - rhoinv[i] * yb[i];
    ldl_solve(&f, rhs, sol, wk);
    /* x update, relaxation */
    for (int j = 0; j < n; ++j) xb[j] = alpha * sol[j] + (1.0 - alpha) * xb[j];
    for (int i = 0; i < m; ++i) {
      /* z-tilde from nu; v = alpha z~ + (1-alpha) z + y/rho; z = Pi(v); y = rho (v - z) */
      double zt = zb[i] + rhoinv[i] * (sol[n + i] - yb[i]);
      double v = alpha * zt + (1.0 - alpha) * zb[i] + rhoinv[i] * yb[i];
      double zn = dmin(dmax(v, w.l[i]), w.u[i]);
      yb[i] = rho[i] * (v - zn);
      zb[i] = zn;
    }
    ++k;
    int check = (s->check_every > 0 && k % s->check_every == 0) || k == s->max_iter;
    if (!check) continue;
    residuals(&w, s, xb, zb, yb, Ax, Px, Aty, &res);
    if (res.prim_res <= res.eps_prim && res.dual_res <= res.eps_dual) {
      status = ORC_SOLVED;
      break;
    }
    for (int j = 0; j < n; ++j) dx[j] = xb[j] - xprev[j];
    for (int i = 0; i < m; ++i) dy[i] = yb[i] - yprev[i];
    if (primal_infeasible(&w, s, dy, Px)) { status = ORC_PRIMAL_INFEASIBLE; break; }
    if (dual_infeasible(&w, s, dx, Px, Ax)) { status = ORC_DUAL_INFEASIBLE; break; }
    if (s->time_limit > 0.0 && now_s() - t0 >= s->time_limit) {
      status = ORC_TIME_LIMIT_REACHED;
      break;
    }
    if (k == s->max_iter) { status = ORC_MAX_ITER_REACHED; break; }
    if (s->adaptive_rho) {
      /* Section 5.2 rho-bar rule on the scaled residuals, at every check */
      {
        double rnew = orc_rho_update(rho_bar, res.prim_res_s, res.prim_norm_s, res.dual_res_s,
                                     res.dual_norm_s);
        if (rnew != rho_bar) {
          rho_bar = rnew;
          set_rho(&w, pb->l, pb->u, rho_bar, rho, rhoinv);
          for (int i = 0; i < m; ++i) K.Kx[K.diag_pos[n + i]] = -rhoinv[i];
          rc = ldl_numeric(&f, K.Kp, K.Kx);   /* new numeric factorisation only */
          if (rc != 0) break;
          info->rho_updates++;
        }
      }
    }
  }
  if (k == 0) status = ORC_MAX_ITER_REACHED;
  double t2 = now_s();
  info->solve_time = t2 - t1;

  info->polish_status = 0;
  if (rc == 0 && status == ORC_SOLVED && s->polish) {
    resid_t admm = res;
    info->polish_status = polish(&w, s, xb, zb, yb, &res, &admm);
  }
  info->polish_time = now_s() - t2;

  /* unscale (Section 5.1): x = D xbar, y = c^-1 E ybar, z = E^-1 zbar */
  double cinv = 1.0 / w.c;
  if (status == ORC_PRIMAL_INFEASIBLE) {
    for (int i = 0; i < m; ++i) y_out[i] = cinv * w.E[i] * dy[i];   /* certificate */
    for (int j = 0; j < n; ++j) x_out[j] = w.D[j] * xb[j];
  } else if (status == ORC_DUAL_INFEASIBLE) {
    for (int j = 0; j < n; ++j) x_out[j] = w.D[j] * dx[j];           /* certificate */
    for (int i = 0; i < m; ++i) y_out[i] = cinv * w.E[i] * yb[i];
  } else {
    for (int j = 0; j < n; ++j) x_out[j] = w.D[j] * xb[j];
    for (int i = 0; i < m; ++i) y_out[i] = cinv * w.E[i] * yb[i];
  }
  for (int i = 0; i < m; ++i) z_out[i] = w.Einv[i] * zb[i];

  /* objective on the original data */
  if (status == ORC_PRIMAL_INFEASIBLE) info->obj_val = INFINITY;
  else if (status == ORC_DUAL_INFEASIBLE) info->obj_val = -INFINITY;
  else {
    double *Pxo = (double *)xmalloc(sizeof(double) * (size_t)n);
    sym_matvec(n, pb->P_indptr, pb->P_indices, pb->P_data, x_out, Pxo);
    double ob = 0.0;
    for (int j = 0; j < n; ++j) ob += 0.5 * x_out[j] * Pxo[j] + pb->q[j] * x_out[j];
    info->obj_val = ob;
    free(Pxo);
  }
  info->status = status;
  info->iter = k;
  info->prim_res = res.prim_res;
  info->dual_res = res.dual_res;
  info->eps_prim = res.eps_prim;
  info->eps_dual = res.eps_dual;
  info->rho_bar = rho_bar;

  ldl_free(&f); kkt_free(&K); wq_free(&w);
  free(rho); free(rhoinv); free(allrows); free(dc);
  free(xb); free(zb); free(yb); free(xprev); free(yprev); free(rhs); free(sol); free(wk);
  free(Ax); free(Px); free(Aty); free(dx); free(dy);
  return rc;
}
