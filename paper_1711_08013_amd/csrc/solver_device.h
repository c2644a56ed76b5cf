// Device side of osqp_mi: per-QP routines written once against a Team
// (workgroup or whole grid) and a working precision T (double for the FP64
// path, float for the mixed path).  Paper references: Algorithm 1 and the
// reduced (indirect) linear system of Section 3.1; termination and
// infeasibility tests of Sections 3.4 and 5.1; modified Ruiz equilibration
// (Section 5.1); rho vector and rho-bar rule (Section 5.2).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dense.h"
#include "qp_layout.h"
#include "team.h"

namespace osqpmi {

// View of one QP inside a packed batch.
template <class T>
struct QPView {
  int n, m, lm, ln;
  const int *arp, *aci, *atrp, *atci, *prp, *pci;
  const double *araw, *atraw, *praw, *qraw, *lraw, *uraw;
  T *av, *atv, *pv, *q, *l, *u, *pdiag;
  double *a64, *at64, *p64, *q64, *l64, *u64;
  double *D, *E, *Dinv, *Einv;
  const unsigned char *iseq;
  T *rho, *rhoinv, *minv;
  double *x, *z, *y, *xt;
  T *zt, *r, *d, *p, *w, *t, *s;
  double *dx, *dy;
  double *zt64, *s64;   // A x~ and the step vector in double (alias zt, s in FP64)
  const double *xws, *yws;
  double *xo, *yo, *zo;
  QPState *st;
  T *L;              // dense factor (row-major, lower), when dense == 1
  T *Linv;           // inverses of its 64 x 64 diagonal blocks (after L)
  double *lr;        // low-rank block (lr_layout), when dense == 2; the band
                     // block (band_layout), when dense == 3
  int ld, dense, mr_cnt;
  const int *mrows;
  const int *bperm, *biperm;   // band ordering: position -> variable, inverse

  __device__ __forceinline__ QPView(const Batch<T> &b, int k) {
    const QPDesc &ds = b.desc[k];
    n = ds.n; m = ds.m; lm = ds.lm; ln = ds.ln;
    arp = b.a_rp + ds.a_rp; aci = b.a_ci + ds.a_nz;
    atrp = b.at_rp + ds.at_rp; atci = b.at_ci + ds.at_nz;
    prp = b.p_rp + ds.p_rp; pci = b.p_ci + ds.p_nz;
    araw = b.a_raw + ds.a_nz; atraw = b.at_raw + ds.at_nz; praw = b.p_raw + ds.p_nz;
    qraw = b.q_raw + ds.xo; lraw = b.l_raw + ds.yo; uraw = b.u_raw + ds.yo;
    av = b.a_v + ds.a_nz; atv = b.at_v + ds.at_nz; pv = b.p_v + ds.p_nz;
    q = b.q + ds.xo; l = b.l + ds.yo; u = b.u + ds.yo; pdiag = b.pdiag + ds.xo;
    a64 = b.a64 + ds.a_nz; at64 = b.at64 + ds.at_nz; p64 = b.p64 + ds.p_nz;
    q64 = b.q64 + ds.xo; l64 = b.l64 + ds.yo; u64 = b.u64 + ds.yo;
    D = b.D + ds.xo; E = b.E + ds.yo; Dinv = b.Dinv + ds.xo; Einv = b.Einv + ds.yo;
    iseq = b.is_eq + ds.yo;
    rho = b.rho + ds.yo; rhoinv = b.rhoinv + ds.yo; minv = b.minv + ds.xo;
    x = b.x + ds.xo; z = b.z + ds.yo; y = b.y + ds.yo; xt = b.xt + ds.xo; zt = b.zt + ds.yo;
    r = b.r + ds.xo; d = b.d + ds.xo; p = b.p + ds.xo; w = b.w + ds.xo;
    t = b.t + ds.yo; s = b.s + ds.yo;
    dx = b.dx + ds.xo; dy = b.dy + ds.yo;
    zt64 = b.zt64 + ds.yo; s64 = b.s64 + ds.yo;
    xws = b.xws + ds.xo; yws = b.yws + ds.yo;
    xo = b.xo + ds.xo; yo = b.yo + ds.yo; zo = b.zo + ds.yo;
    st = b.st + k;
    dense = ds.dense; ld = ds.dld; mr_cnt = ds.mr_cnt;
    L = ds.dense == 1 ? b.dmat + ds.dense_off : nullptr;
    Linv = ds.dense == 1 ? L + (size_t)ds.n * ds.dld : nullptr;
    lr = (ds.dense == 2 || ds.dense == 3) ? b.lmat + ds.dense_off : nullptr;
    mrows = b.mrows + ds.mr_off;
    bperm = b.bperm + ds.xo; biperm = b.biperm + ds.xo;
  }
};

// Row-group mapping: aligned groups of L lanes walk the rows of a pass.
struct Rows {
  int g, lane, ng, L;
  template <class Team>
  __device__ __forceinline__ Rows(const Team &tm, int L_) : L(L_) {
    g = tm.tid / L; lane = tm.tid & (L - 1); ng = tm.nt / L;
  }
};

// Partial dot over the lanes of a group of sum_k v[k] x[ci[k]], k in [b, e)
// (not reduced).  Each round gathers eight entries per lane, all in flight
// together: the passes are bound by memory latency per wave, not by
// arithmetic, and a row needs ceil(len / 8L) rounds.
template <class A, class V, class X>
__device__ __forceinline__ A seg_partial(const int *ci, const V *v, int b, int e, int lane, int L,
                                         const X *x) {
  A s0 = A(0), s1 = A(0), s2 = A(0), s3 = A(0);
  for (int k = b + lane; k < e; k += 8 * L) {
    int c[8];
    A a[8];
    // positions past the row's end re-read its last entry (always in
    // range, since k < e) and contribute zero: the loads stay unconditional,
    // so none of them waits for another
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kk = min(k + u * L, e - 1);
      c[u] = ci[kk];
      a[u] = A(v[kk]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k + u * L >= e) a[u] = A(0);
    s0 += a[0] * A(x[c[0]]); s1 += a[1] * A(x[c[1]]);
    s2 += a[2] * A(x[c[2]]); s3 += a[3] * A(x[c[3]]);
    s0 += a[4] * A(x[c[4]]); s1 += a[5] * A(x[c[5]]);
    s2 += a[6] * A(x[c[6]]); s3 += a[7] * A(x[c[7]]);
  }
  return (s0 + s1) + (s2 + s3);
}

// Four consecutive entries from a 16-byte-aligned address.
__device__ __forceinline__ void ld4(const int *p, int (&o)[4]) {
  const int4 t = *reinterpret_cast<const int4 *>(p);
  o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
}
__device__ __forceinline__ void ld4(const float *p, float (&o)[4]) {
  const float4 t = *reinterpret_cast<const float4 *>(p);
  o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
}
__device__ __forceinline__ void ld4(const double *p, double (&o)[4]) {
  const double2 t0 = *reinterpret_cast<const double2 *>(p);
  const double2 t1 = *reinterpret_cast<const double2 *>(p + 2);
  o[0] = t0.x; o[1] = t0.y; o[2] = t1.x; o[3] = t1.y;
}

// seg_partial with 16-byte loads: each lane takes aligned chunks of four
// consecutive entries (the entry arrays of a QP start on a multiple of 4 and
// are padded to one), four chunks per round.  Entries of a chunk outside
// [b, e) are masked; a chunk past the row's end re-reads the row's last
// chunk, which is in range, so every load is unconditional.
template <class A, class V, class X>
__device__ __forceinline__ A seg_partial4(const int *ci, const V *v, int b, int e, int lane,
                                          int L, const X *x) {
  A s0 = A(0), s1 = A(0), s2 = A(0), s3 = A(0);
  if (e <= b) return A(0);
  const int last = (e - 1) & ~3;
  for (int k = (b & ~3) + 4 * lane; k < e; k += 16 * L) {
    int c[4][4];
    V a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(k + 4 * L * u, last);
      ld4(ci + kk, c[u]);
      ld4(v + kk, a[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * L * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool ok = kk + q >= b && kk + q < e;
        const int cq = ok ? c[u][q] : 0;
        const A aq = ok ? A(a[u][q]) : A(0);
        const A t = aq * A(x[cq]);
        if (q == 0) s0 += t; else if (q == 1) s1 += t; else if (q == 2) s2 += t; else s3 += t;
      }
    }
  }
  return (s0 + s1) + (s2 + s3);
}

// seg_partial4 against two gathered vectors at once (one pass over the
// entries): .x = sum v[k] x[ci[k]], .y = sum v[k] y[ci[k]], each in
// seg_partial4's order.
template <class V>
__device__ __forceinline__ double2 seg_partial4x2(const int *ci, const V *v, int b, int e, int lane,
                                                  int L, const double *x, const double *y) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
  if (e <= b) return double2{0.0, 0.0};
  const int last = (e - 1) & ~3;
  for (int k = (b & ~3) + 4 * lane; k < e; k += 16 * L) {
    int c[4][4];
    V a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(k + 4 * L * u, last);
      ld4(ci + kk, c[u]);
      ld4(v + kk, a[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * L * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool ok = kk + q >= b && kk + q < e;
        const int cq = ok ? c[u][q] : 0;
        const double aq = ok ? double(a[u][q]) : 0.0;
        const double tx = aq * x[cq], ty = aq * y[cq];
        if (q == 0) { s0 += tx; t0 += ty; }
        else if (q == 1) { s1 += tx; t1 += ty; }
        else if (q == 2) { s2 += tx; t2 += ty; }
        else { s3 += tx; t3 += ty; }
      }
    }
  }
  return double2{(s0 + s1) + (s2 + s3), (t0 + t1) + (t2 + t3)};
}

// sum over [b, e) of f(v[k], ci[k]) for the lanes of a group (not reduced),
// with seg_partial4's chunked unconditional loads and summation order.
template <class A, class V, class F>
__device__ __forceinline__ A seg_sum4(const int *ci, const V *v, int b, int e, int lane, int L,
                                      F &&f) {
  A s0 = A(0), s1 = A(0), s2 = A(0), s3 = A(0);
  if (e <= b) return A(0);
  const int last = (e - 1) & ~3;
  for (int k = (b & ~3) + 4 * lane; k < e; k += 16 * L) {
    int c[4][4];
    V a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(k + 4 * L * u, last);
      ld4(ci + kk, c[u]);
      ld4(v + kk, a[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * L * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool ok = kk + q >= b && kk + q < e;
        const A t = ok ? f(A(a[u][q]), c[u][q]) : A(0);
        if (q == 0) s0 += t; else if (q == 1) s1 += t; else if (q == 2) s2 += t; else s3 += t;
      }
    }
  }
  return (s0 + s1) + (s2 + s3);
}

// f(ci[k], v[k]) for every k in [b, e) on the lanes of a group, with the
// chunked unconditional loads of seg_partial4.
template <class V, class F>
__device__ __forceinline__ void seg_each4(const int *ci, const V *v, int b, int e, int lane, int L,
                                          F &&f) {
  if (e <= b) return;
  const int last = (e - 1) & ~3;
  for (int k = (b & ~3) + 4 * lane; k < e; k += 16 * L) {
    int c[4][4];
    V a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(k + 4 * L * u, last);
      ld4(ci + kk, c[u]);
      ld4(v + kk, a[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * L * u;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (kk + q >= b && kk + q < e) f(c[u][q], a[u][q]);
    }
  }
}


// Rows t = g, g + ng, ... < cnt (CSR row rowof(t)); per lane group of L
// lanes, sum over the row of v[k] x[ci[k]], then epi(t, i, sum, pre) with
// pre = pro(i) loaded when the row became current.  The chunk loads of the
// next round (of this row or of the next) are issued before the current
// round's gathers; the summation order is seg_partial4's.
template <class A, class V, class X, class RowOf, class Pro, class Epi>
__device__ __forceinline__ void stream_rows(const int *rp, const int *ci, const V *v, const X *x,
                                            int g, int ng, int cnt, int lane, int L, RowOf &&rowof,
                                            Pro &&pro, Epi &&epi) {
  int t = g;
  int i = t < cnt ? rowof(t) : 0;
  int b = t < cnt ? rp[i] : 0, e = t < cnt ? rp[i + 1] : 0;
  int t2 = t + ng;
  int i2 = t2 < cnt ? rowof(t2) : 0;
  int b2 = t2 < cnt ? rp[i2] : 0, e2 = t2 < cnt ? rp[i2 + 1] : 0;
  decltype(pro(0)) pre{};
  if (t < cnt) pre = pro(i);
  int kb = b & ~3;   // round base, the same for every lane of the group
  int c[4][4];
  V a[4][4];
  auto load = [&](int kp, int bb, int eb, int (&cc)[4][4], V (&aa)[4][4]) __attribute__((always_inline)) {
    if (eb <= bb) {   // empty row: nothing to read (its start may be the array's end)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) { cc[u][q] = 0; aa[u][q] = V(0); }
      return;
    }
    const int last = (eb - 1) & ~3;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(kp + 4 * L * u, last);
      ld4(ci + kk, cc[u]);
      ld4(v + kk, aa[u]);
    }
  };
  if (t < cnt) load(kb + 4 * lane, b, e, c, a);
  A s0 = A(0), s1 = A(0), s2 = A(0), s3 = A(0);
  while (t < cnt) {
    const bool same = kb + 16 * L < e;   // uniform in the group
    const int kbn = same ? kb + 16 * L : (b2 & ~3);
    const int bn = same ? b : b2, en = same ? e : e2;
    const bool more = same || t2 < cnt;
    int cn[4][4];
    V an[4][4];
    if (more) load(kbn + 4 * lane, bn, en, cn, an);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = kb + 4 * lane + 4 * L * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool ok = kk + q >= b && kk + q < e;
        const int cq = ok ? c[u][q] : 0;
        const A aq = ok ? A(a[u][q]) : A(0);
        const A tq = aq * A(x[cq]);
        if (q == 0) s0 += tq; else if (q == 1) s1 += tq; else if (q == 2) s2 += tq; else s3 += tq;
      }
    }
    if (!same) {
      const A sum = group_sum((s0 + s1) + (s2 + s3), L);
      epi(t, i, sum, pre);
      s0 = s1 = s2 = s3 = A(0);
      const int t3 = t2 + ng;
      const int i3 = t3 < cnt ? rowof(t3) : 0;
      const int b3 = t3 < cnt ? rp[i3] : 0, e3 = t3 < cnt ? rp[i3 + 1] : 0;
      t = t2; i = i2; b = b2; e = e2;
      t2 = t3; i2 = i3; b2 = b3; e2 = e3;
      if (t < cnt) pre = pro(i);
    }
    kb = kbn;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) { c[u][q] = cn[u][q]; a[u][q] = an[u][q]; }
  }
}

// max_k |v[k]| s[ci[k]] over [b, e) for the lanes of a group (not reduced),
// with the chunked unconditional loads of seg_chunks.
template <class S>
__device__ __forceinline__ double seg_absmax4(const int *ci, const double *v, int b, int e, int lane,
                                              int L, const S *sc) {
  double m0 = 0.0, m1 = 0.0;
  if (e <= b) return 0.0;
  const int last = (e - 1) & ~3;
  for (int k = (b & ~3) + 4 * lane; k < e; k += 16 * L) {
    int c[4][4];
    double a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(k + 4 * L * u, last);
      ld4(ci + kk, c[u]);
      ld4(v + kk, a[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 4 * L * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool ok = kk + q >= b && kk + q < e;
        const double t = ok ? fabs(a[u][q]) * double(sc[ok ? c[u][q] : 0]) : 0.0;
        if (q & 1) m1 = fmax(m1, t); else m0 = fmax(m0, t);
      }
    }
  }
  return fmax(m0, m1);
}

// The same for CSR row r.
template <class A, class V, class X>
__device__ __forceinline__ A row_partial(const int *rp, const int *ci, const V *v, int r,
                                         int lane, int L, const X *x) {
  return seg_partial4<A>(ci, v, rp[r], rp[r + 1], lane, L, x);
}

// Rows j = g, g + ng, ... < cnt of one CSR (rp) or of two with the same row
// count (rp, rp2): f(j, b, e[, b2, e2]) gets the row bounds, which were
// loaded one step ahead so that their latency hides behind the previous row.
template <class F>
__device__ __forceinline__ void rows_ahead(const int *rp, int g, int ng, int cnt, F &&f) {
  int j = g;
  int b = j < cnt ? rp[j] : 0, e = j < cnt ? rp[j + 1] : 0;
  while (j < cnt) {
    const int jn = j + ng;
    const int bn = jn < cnt ? rp[jn] : 0, en = jn < cnt ? rp[jn + 1] : 0;
    f(j, b, e);
    j = jn; b = bn; e = en;
  }
}
template <class F>
__device__ __forceinline__ void rows_ahead2(const int *rp, const int *rp2, int g, int ng, int cnt,
                                            F &&f) {
  int j = g;
  int b = 0, e = 0, b2 = 0, e2 = 0;
  if (j < cnt) { b = rp[j]; e = rp[j + 1]; b2 = rp2[j]; e2 = rp2[j + 1]; }
  while (j < cnt) {
    const int jn = j + ng;
    int bn = 0, en = 0, bn2 = 0, en2 = 0;
    if (jn < cnt) { bn = rp[jn]; en = rp[jn + 1]; bn2 = rp2[jn]; en2 = rp2[jn + 1]; }
    f(j, b, e, b2, e2);
    j = jn; b = bn; e = en; b2 = bn2; e2 = en2;
  }
}

// A pass over the rows of A: rows with at most one entry take one lane each,
// the rows with several entries (the list mrows) a group of rm.L lanes, the
// next row's index and bounds loaded ahead.  body(i, b, e, lane, L) reduces
// over its L lanes; lane 0 holds the result.
template <class T, class Team, class Body>
__device__ __forceinline__ void for_a_rows(const Team &tm, const QPView<T> &v, const Rows &rm,
                                           Body &&body) {
  for (int i = tm.tid; i < v.m; i += tm.nt) {
    const int b = v.arp[i], e = v.arp[i + 1];
    if (e - b <= 1) body(i, b, e, 0, 1);
  }
  const int cnt = v.mr_cnt, ng = rm.ng;
  int r = rm.g;
  int i = r < cnt ? v.mrows[r] : 0;
  int b = r < cnt ? v.arp[i] : 0, e = r < cnt ? v.arp[i + 1] : 0;
  int r2 = r + ng;
  int i2 = r2 < cnt ? v.mrows[r2] : 0;
  while (r < cnt) {
    const int r3 = r2 + ng;
    const int i3 = r3 < cnt ? v.mrows[r3] : 0;
    const int b2 = r2 < cnt ? v.arp[i2] : 0, e2 = r2 < cnt ? v.arp[i2 + 1] : 0;
    body(i, b, e, rm.lane, rm.L);
    r = r2; i = i2; b = b2; e = e2; r2 = r3; i2 = i3;
  }
}

__device__ __forceinline__ double clamp_norm(double v) {
  // reading: a column norm below 1e-4 counts as 1, above 1e4 as 1e4
  return v < 1e-4 ? 1.0 : (v > 1e4 ? 1e4 : v);
}

// Scaled A entry; A and A' rows use this one expression so their values
// stay bit-identical.
__device__ __forceinline__ double scale_a(double raw, double Ei, double Dj) {
  return (raw * Ei) * Dj;
}

// ------------------------------------------------------------------------
// Modified Ruiz equilibration on the device (Section 5.1), from the
// resident unscaled data; then writes the scaled data in T and in double.
// ------------------------------------------------------------------------
template <class T, class Team>
__device__ __forceinline__ void scale_qp(const Team &tm, const QPView<T> &v, const DevSettings &set,
                                         double *stage = nullptr) {
  const int n = v.n, m = v.m;
  // D and E live in LDS during the passes when they fit (the norms gather
  // from them), in global memory otherwise
  const int n8 = (n + 7) & ~7;
  const bool stg = stage != nullptr && n8 + ((m + 7) & ~7) <= kStage;
  double *Dv = stg ? stage : v.D, *Ev = stg ? stage + n8 : v.E;
  for (int j = tm.tid; j < n; j += tm.nt) Dv[j] = 1.0;
  for (int i = tm.tid; i < m; i += tm.nt) Ev[i] = 1.0;
  double c = 1.0;
  tm.sync();
  const Rows rn(tm, v.ln), rm(tm, v.lm);
  auto passes = [&](double *Ds, double *Es) __attribute__((always_inline)) {
    for (int it = 0; it < set.scaling_iters; ++it) {
      // column infinity norms of M = [P A'; A 0] (current scaling) -> delta
      rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n,
                  [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
        const double Dj = Ds[j];
        double a = c * seg_absmax4(v.pci, v.praw, pb, pe, rn.lane, rn.L, Ds);
        a = fmax(a, seg_absmax4(v.atci, v.atraw, ab, ae, rn.lane, rn.L, Es));
        a = group_max(a, rn.L) * Dj;
        if (rn.lane == 0) v.dx[j] = 1.0 / sqrt(clamp_norm(a));
      });
      for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
        const double Ei = Es[i];
        double a = seg_absmax4(v.aci, v.araw, b, e, lane, L, Ds);
        a = group_max(a, L) * Ei;
        if (lane == 0) v.dy[i] = 1.0 / sqrt(clamp_norm(a));
      });
      tm.sync();
      for (int j = tm.tid; j < n; j += tm.nt) Ds[j] *= v.dx[j];
      for (int i = tm.tid; i < m; i += tm.nt) Es[i] *= v.dy[i];
      tm.sync();
      // cost scaling: gamma = 1 / max(mean_j ||Pbar_j||_inf, ||qbar||_inf)
      double red[2] = {0.0, 0.0};
      rows_ahead(v.prp, rn.g, rn.ng, n, [&](int j, int pb, int pe) __attribute__((always_inline)) {
        const double Dj = Ds[j], qj = v.qraw[j];
        double a = seg_absmax4(v.pci, v.praw, pb, pe, rn.lane, rn.L, Ds);
        a = group_max(a, rn.L) * (c * Dj);
        if (rn.lane == 0) {
          red[0] += a;
          red[1] = fmax(red[1], fabs(c * Dj * qj));
        }
      });
      tm.template reduce<1, 1>(red);
      const double s = fmax(red[0] / (double)n, red[1]);
      // reading: gamma = 1 when P and q vanish, else clamped to [1e-4, 1e4]
      const double gamma = s == 0.0 ? 1.0 : fmin(fmax(1.0 / s, 1e-4), 1e4);
      c *= gamma;
    }
  };
  if (stg) {
    passes(stage, stage + n8);
    for (int j = tm.tid; j < n; j += tm.nt) v.D[j] = stage[j];
    for (int i = tm.tid; i < m; i += tm.nt) v.E[i] = stage[n8 + i];
    tm.sync();
  } else {
    passes(v.D, v.E);
  }
  // write the scaled problem: Pbar = c D P D, qbar = c D q, Abar = E A D,
  // lbar = E l, ubar = E u
  // (columns of P without a diagonal entry keep pdiag = 0)
  for (int j = tm.tid; j < n; j += tm.nt) {
    const double Dj = v.D[j];
    const double qq = c * Dj * v.qraw[j];
    v.q64[j] = qq;
    v.q[j] = T(qq);
    v.Dinv[j] = 1.0 / Dj;
    v.pdiag[j] = T(0);
  }
  for (int i = tm.tid; i < m; i += tm.nt) {
    const double Ei = v.E[i];
    const double lo = v.lraw[i] * Ei, hi = v.uraw[i] * Ei;
    v.l64[i] = lo; v.u64[i] = hi;
    v.l[i] = T(lo); v.u[i] = T(hi);
    v.Einv[i] = 1.0 / Ei;
  }
  tm.sync();
  rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n,
              [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
    const double Dj = v.D[j];
    for (int k = pb + rn.lane; k < pe; k += rn.L) {
      const double val = c * (v.praw[k] * Dj) * v.D[v.pci[k]];
      v.p64[k] = val;
      v.pv[k] = T(val);
      if (v.pci[k] == j) v.pdiag[j] = T(val);
    }
    for (int k = ab + rn.lane; k < ae; k += rn.L) {
      const double val = scale_a(v.atraw[k], v.E[v.atci[k]], Dj);
      v.at64[k] = val;
      v.atv[k] = T(val);
    }
  });
  for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
    const double Ei = v.E[i];
    for (int k = b + lane; k < e; k += L) {
      const double val = scale_a(v.araw[k], Ei, v.D[v.aci[k]]);
      v.a64[k] = val;
      v.av[k] = T(val);
    }
  });
  if (tm.tid == 0) v.st->c = c;
  tm.sync();
}

// Rescale new vectors (q, l, u) with the stored D, E, c (Section 6).
template <class T, class Team>
__device__ __forceinline__ void rescale_vectors(const Team &tm, const QPView<T> &v) {
  const double c = v.st->c;
  for (int j = tm.tid; j < v.n; j += tm.nt) {
    const double qq = c * v.D[j] * v.qraw[j];
    v.q64[j] = qq; v.q[j] = T(qq);
  }
  for (int i = tm.tid; i < v.m; i += tm.nt) {
    const double lo = v.lraw[i] * v.E[i], hi = v.uraw[i] * v.E[i];
    v.l64[i] = lo; v.u64[i] = hi; v.l[i] = T(lo); v.u[i] = T(hi);
  }
  tm.sync();
}

// rho_i = rho-bar (l_i != u_i) or 1e3 rho-bar (l_i == u_i), Section 5.2;
// Jacobi preconditioner of P + sigma I + A' R A: diag(P) + sigma + sum_i rho_i A_ij^2.
template <class T, class Team>
__device__ __forceinline__ void set_rho_and_precond(const Team &tm, const QPView<T> &v, double rho_bar,
                                    double sigma) {
  for (int i = tm.tid; i < v.m; i += tm.nt) {
    const double r = v.iseq[i] ? 1e3 * rho_bar : rho_bar;
    v.rho[i] = T(r);
    v.rhoinv[i] = T(1.0 / r);
  }
  tm.sync();
  const Rows rn(tm, v.ln);
  for (int j = rn.g; j < v.n; j += rn.ng) {
    double a = 0.0;
    for (int k = v.atrp[j] + rn.lane; k < v.atrp[j + 1]; k += rn.L) {
      const double e = v.at64[k];
      a += (double)v.rho[v.atci[k]] * e * e;
    }
    a = group_sum(a, rn.L);
    if (rn.lane == 0) v.minv[j] = T(1.0 / ((double)v.pdiag[j] + sigma + a));
  }
  tm.sync();
}

// ------------------------------------------------------------------------
// Dense path: form Kbar = P + sigma I + A' R A (rows of A with one entry
// add to the diagonal, the others through the rank-k update B'B with
// B = R^1/2 A restricted to them) and factor it, Kbar = L L'.
// ------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool form_and_factor(const WGTeam &tm, const QPView<T> &v, DenseLDS<T> &s, T *B,
                                double sigma) {
  const int n = v.n, ld = v.ld, R = v.mr_cnt;
  for (size_t e = tm.tid; e < (size_t)n * ld; e += tm.nt) v.L[e] = T(0);
  for (size_t e = tm.tid; e < (size_t)R * n; e += tm.nt) B[e] = T(0);
  tm.sync();
  for (int j = tm.tid; j < n; j += tm.nt) {
    for (int k = v.prp[j]; k < v.prp[j + 1]; ++k) {
      const int c = v.pci[k];
      if (c <= j) v.L[(size_t)j * ld + c] = v.pv[k];
    }
    T dsum = T(sigma);
    for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) {
      const int i = v.atci[k];
      if (v.arp[i + 1] - v.arp[i] == 1) dsum += v.rho[i] * v.atv[k] * v.atv[k];
    }
    v.L[(size_t)j * ld + j] += dsum;
  }
  for (int r = tm.tid; r < R; r += tm.nt) {
    const int i = v.mrows[r];
    const T sr = T(sqrt(double(v.rho[i])));
    for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) B[(size_t)r * n + v.aci[k]] = sr * v.av[k];
  }
  tm.sync();
  dense_syrk_tn<T>(tm, s, v.L, ld, B, n, R, n, T(1));
  const bool ok = dense_cholesky<T>(tm, s, v.L, ld, n);
  if (ok) dense_invert_diag<T>(tm, s, v.L, ld, n, v.Linv);
  return ok;
}

// d = (L L')^-1 r
template <class T>
__device__ __forceinline__ void precondition_dense(const WGTeam &tm, const QPView<T> &v, DenseLDS<T> &s) {
  tm.sync();
  for (int j = tm.tid; j < v.n; j += tm.nt) v.d[j] = v.r[j];
  tm.sync();
  dense_solve_llt<T>(tm, s, v.L, v.ld, v.n, v.Linv, v.d);
}

// ------------------------------------------------------------------------
// Band path (dense == 3).  With the ordering found on the host (bperm:
// position -> variable), the permuted reduced matrix
//     Kp = (P + sigma I + A'RA)[bperm, bperm]
// has half-bandwidth at most nb, so in nb x nb blocks it is block
// tridiagonal: diagonal blocks A_i and sub-diagonal blocks B_i (rows of
// block i+1, columns of block i).  Its Cholesky factor is block bidiagonal:
// with D_0 = A_0,
//     L_ii L_ii' = D_i,   C_i = B_i L_ii^-T,   D_{i+1} = A_{i+1} - C_i C_i',
// and C_i is upper triangular (B_i is, since the band ends within nb of the
// diagonal, and L_ii^-T is).  Stored per block row, in FP64: Linv_i = L_ii^-1
// and C_i.  A solve is a forward sweep y_i = Linv_i (z_i - C_{i-1} y_{i-1})
// and a backward sweep x_i = Linv_i' (y_i - C_i' x_{i+1}): O(n nb) work and
// bytes instead of the dense factor's O(n^2).  This is the direct method of
// Section 3.1 on the reduced system: the symbolic step (the fill-limiting
// ordering) on the host, the numeric step per QP here, redone on a rho-bar
// change, and every ADMM step takes x~ += Kp^-1 r in FP64 (the matrix values
// are the working-precision copies the other passes use, so the factor is
// exact for the same K).
// ------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool band_form_and_factor(const WGTeam &tm, const QPView<T> &v,
                                                     DenseLDS<double> &s, double *W,
                                                     double sigma, double rho_bar) {
  const int n = v.n, nb = v.ld, nblk = (n + nb - 1) / nb, nb2 = nb * nb;
  const BandLayout bl = band_layout(n, nb);
  const BandScratch ws = band_scratch_layout(nb);
  double *F = v.lr + bl.tiles;
  double *D = W + ws.D, *Bp = W + ws.Bp, *X = W + ws.X;
  const int sw = 2 * nb;   // strip row length: columns i0 - nb .. i0 + nb - 1
  for (int i = 0; i < nblk; ++i) {
    const int i0 = i * nb, ni = min(nb, n - i0), qlo = i0 - nb;
    // (1) strip of rows i0 .. i0 + ni - 1, columns qlo .. row (the lower part
    //     of the band): kBandCopies lanes per row, lane c accumulating every
    //     c-th term into its own copy (fixed order, no atomics)
    for (int e = tm.tid; e < kBandCopies * nb * sw; e += tm.nt) W[ws.strip + e] = 0.0;
    tm.sync();
    for (int t = tm.tid; t < nb * kBandCopies; t += tm.nt) {
      const int a = t / kBandCopies, c = t % kBandCopies;
      if (a >= ni) continue;
      const int p = i0 + a, j = v.bperm[p];
      double *row = W + ws.strip + (size_t)c * nb * sw + (size_t)a * sw;
      for (int k = v.prp[j] + c; k < v.prp[j + 1]; k += kBandCopies) {
        const int q = v.biperm[v.pci[k]];
        if (q >= qlo && q <= p) row[q - qlo] += double(v.pv[k]);
      }
      if (c == 0) row[p - qlo] += sigma;
      for (int k = v.atrp[j] + c; k < v.atrp[j + 1]; k += kBandCopies) {
        const int r = v.atci[k];
        const double w = (v.iseq[r] ? 1e3 * rho_bar : rho_bar) * double(v.atv[k]);
        for (int e = v.arp[r]; e < v.arp[r + 1]; ++e) {
          const int q = v.biperm[v.aci[e]];
          if (q >= qlo && q <= p) row[q - qlo] += w * double(v.av[e]);
        }
      }
    }
    tm.sync();
    for (int e = tm.tid; e < nb * sw; e += tm.nt) {
      const int a = e / sw, col = e % sw;
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < kBandCopies; ++c) sum += W[ws.strip + (size_t)c * nb * sw + e];
      if (col >= nb) D[a * nb + (col - nb)] = (a < ni && col - nb <= a) ? sum : 0.0;
      else Bp[a * nb + col] = a < ni ? sum : 0.0;
    }
    tm.sync();
    if (i > 0) {
      // (2) C_{i-1} = Bp Linv_{i-1}': C[a][d] = sum_{e <= d} Bp[a][e] Linv[d][e]
      const double *Lp = F + (size_t)(2 * (i - 1)) * nb2;
      double *Cp = F + (size_t)(2 * (i - 1) + 1) * nb2;
      for (int t = tm.tid; t < nb2; t += tm.nt) {
        const int a = t / nb, d = t % nb;
        double acc = 0.0;
        for (int e = 0; e <= d; ++e) acc += Bp[a * nb + e] * Lp[d * nb + e];
        Cp[t] = a < ni ? acc : 0.0;
      }
      tm.sync();
      // (3) D -= C C' (lower triangle)
      for (int t = tm.tid; t < nb2; t += tm.nt) {
        const int a = t / nb, c = t % nb;
        if (a >= ni || c > a) continue;
        double acc = 0.0;
        for (int e = 0; e < nb; ++e) acc += Cp[a * nb + e] * Cp[c * nb + e];
        D[t] -= acc;
      }
      tm.sync();
    }
    // (4) D = L_ii L_ii', then Linv_i = L_ii^-1 (the 64 x 64 inverse tile in X)
    if (!dense_cholesky<double>(tm, s, D, nb, ni)) return false;
    dense_invert_diag<double>(tm, s, D, nb, ni, X);
    double *Li = F + (size_t)(2 * i) * nb2;
    for (int t = tm.tid; t < nb2; t += tm.nt) {
      const int a = t / nb, c = t % nb;
      Li[t] = (a < ni && c < ni) ? X[a * 64 + c] : 0.0;
    }
    tm.sync();
  }
  return true;
}

// The direct step with the band factor: x~ += Kbar^-1 r, r the FP64
// residual the start pass left in the band block (variable order).  z (LDS,
// n doubles) takes r[bperm]; the two sweeps run in place on it; tmp (LDS, 64
// doubles) holds a block's intermediate vector.  Four lanes per row (or
// column) of a tile, each over 16 columns (rows), only the tile's nonzero
// triangle read.
template <class T>
__device__ __forceinline__ void band_direct_step(const WGTeam &tm, const QPView<T> &v, double *z,
                                                 double *tmp) {
  const int n = v.n, nb = v.ld, nblk = (n + nb - 1) / nb, nb2 = nb * nb;
  const BandLayout bl = band_layout(n, nb);
  const double *F = v.lr + bl.tiles, *rv = v.lr + bl.r;
  tm.sync();
  for (int p = tm.tid; p < n; p += tm.nt) z[p] = rv[v.bperm[p]];
  tm.sync();
  // forward: y_i = Linv_i (z_i - C_{i-1} y_{i-1})
  for (int i = 0; i < nblk; ++i) {
    const int i0 = i * nb, ni = min(nb, n - i0);
    const double *Li = F + (size_t)(2 * i) * nb2;
    const double *Cp = i > 0 ? F + (size_t)(2 * (i - 1) + 1) * nb2 : nullptr;
    for (int t = tm.tid; t < nb * 4; t += tm.nt) {
      const int a = t >> 2, part = t & 3;
      double acc = 0.0;
      if (Cp != nullptr && a < ni)
        for (int d = max(a, part * 16); d < min(nb, part * 16 + 16); ++d)
          acc += Cp[a * nb + d] * z[i0 - nb + d];
      acc = group_sum(acc, 4);
      if (part == 0 && a < ni) tmp[a] = z[i0 + a] - acc;
    }
    tm.sync();
    for (int t = tm.tid; t < nb * 4; t += tm.nt) {
      const int a = t >> 2, part = t & 3;
      double acc = 0.0;
      if (a < ni)
        for (int e = part * 16; e < min(a + 1, part * 16 + 16); ++e) acc += Li[a * nb + e] * tmp[e];
      acc = group_sum(acc, 4);
      if (part == 0 && a < ni) z[i0 + a] = acc;
    }
    tm.sync();
  }
  // backward: x_i = Linv_i' (y_i - C_i' x_{i+1})
  for (int i = nblk - 1; i >= 0; --i) {
    const int i0 = i * nb, ni = min(nb, n - i0);
    const double *Li = F + (size_t)(2 * i) * nb2;
    const bool has_next = i + 1 < nblk;
    const double *Ci = has_next ? F + (size_t)(2 * i + 1) * nb2 : nullptr;
    const int n1 = has_next ? min(nb, n - i0 - nb) : 0;
    for (int t = tm.tid; t < nb * 4; t += tm.nt) {
      const int d = t >> 2, part = t & 3;
      double acc = 0.0;
      if (has_next && d < ni)
        for (int a = part * 16; a < min(min(d + 1, n1), part * 16 + 16); ++a)
          acc += Ci[a * nb + d] * z[i0 + nb + a];
      acc = group_sum(acc, 4);
      if (part == 0 && d < ni) tmp[d] = z[i0 + d] - acc;
    }
    tm.sync();
    for (int t = tm.tid; t < nb * 4; t += tm.nt) {
      const int d = t >> 2, part = t & 3;
      double acc = 0.0;
      if (d < ni)
        for (int a = max(d, part * 16); a < min(ni, part * 16 + 16); ++a) acc += Li[a * nb + d] * tmp[a];
      acc = group_sum(acc, 4);
      if (part == 0 && d < ni) z[i0 + d] = acc;
    }
    tm.sync();
  }
  for (int p = tm.tid; p < n; p += tm.nt) v.xt[v.bperm[p]] += z[p];
  tm.sync();
}

// ------------------------------------------------------------------------
// Diagonal-plus-low-rank path (P diagonal).  With the rows of A split into
// single-entry rows and the R multi-entry rows A_m,
//     K = P + sigma I + A'RA = Delta + B'B,   B = R_m^1/2 A_m  (R x n),
// Delta = diag(P) + sigma + sum over single-entry rows of rho_i a_ij^2.
// The Woodbury identity gives K^-1 r = u - Delta^-1 B' S^-1 B u with
// u = Delta^-1 r and the R x R capacitance matrix S = I + B Delta^-1 B',
// formed, factored and inverted once per rho-bar in FP64 (S = G G' + I,
// G = B Delta^-1/2 formed densely in the workgroup's scratch).  This is the
// same reduced system the dense factor solves, at O(R^2 n) set-up and
// O(nnz(A_m) + R^2) per apply.
// ------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ bool lowrank_form_and_factor(const WGTeam &tm, const QPView<T> &v,
                                                        DenseLDS<double> &s, double *G,
                                                        double sigma, double rho_bar) {
  const int n = v.n, m = v.m, R = v.mr_cnt, ldS = v.ld, ldg = (n + 7) & ~7;
  const LRLayout lo = lr_layout(n, m, R, ldS);
  double *dinv = v.lr, *S = v.lr + lo.S, *wr = v.lr + lo.wr;
  auto rho_i = [&](int i) -> double { return v.iseq[i] ? 1e3 * rho_bar : rho_bar; };
  // rho_i of the single-entry rows (0 for the others) in w's by-row slots,
  // so that Delta is a gathered sum over the rows of A'
  for (int i = tm.tid; i < m; i += tm.nt) wr[i] = v.arp[i + 1] - v.arp[i] == 1 ? rho_i(i) : 0.0;
  for (size_t e = tm.tid; e < (size_t)R * ldg; e += tm.nt) G[e] = 0.0;
  tm.sync();
  const Rows rn(tm, v.ln);
  rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n, [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
    double a = 0.0;
    for (int k = pb + rn.lane; k < pe; k += rn.L)   // P is diagonal here
      if (v.pci[k] == j) a += double(v.pv[k]);
    a += seg_sum4<double>(v.atci, v.atv, ab, ae, rn.lane, rn.L,
                          [&](double e, int i) __attribute__((always_inline)) { return wr[i] * e * e; });
    a = group_sum(a, rn.L);
    if (rn.lane == 0) dinv[j] = 1.0 / (sigma + a);
  });
  tm.sync();
  for (int i = tm.tid; i < m; i += tm.nt) wr[i] = 0.0;   // single-entry rows stay 0
  const Rows rm(tm, v.lm);
  for (int r = rm.g; r < R; r += rm.ng) {
    const int i = v.mrows[r];
    const double sr = sqrt(rho_i(i));
    seg_each4(v.aci, v.av, v.arp[i], v.arp[i + 1], rm.lane, rm.L,
              [&](int j, T a) __attribute__((always_inline)) {
                G[(size_t)r * ldg + j] = sr * double(a) * sqrt(dinv[j]);
              });
  }
  tm.sync();
  dense_gram_lower(tm, s, G, ldg, R, n, S, ldS);
  for (int r = tm.tid; r < R; r += tm.nt) S[(size_t)r * ldS + r] += 1.0;
  tm.sync();
  const bool ok = dense_cholesky<double>(tm, s, S, ldS, R);
  // S^-1 explicitly (G, no longer needed, is the scratch): each application
  // is then one dense matrix-vector product instead of two block sweeps
  if (ok) dense_spd_inverse(tm, s, S, ldS, R, G, G + (size_t)R * ldS);
  return ok;
}

// K^-1 r by the Woodbury identity, FP64 inside (the matrix values are the
// working-precision copies the other passes use, so the inverse is exact for
// the same K).  u = Delta^-1 r is formed here from r (T), or was left in the
// block's u by the caller (u_ready, from the FP64 residual).  The result goes
// to d (rounded to T) or, to_xt, is added to the FP64 iterate x~ (the direct
// solve).  With an LDS stage (u and the scattered w in LDS) the gathers of
// both sparse passes hit LDS.
template <class T>
__device__ __forceinline__ void precondition_lowrank(const WGTeam &tm, const QPView<T> &v,
                                                     double rho_bar, double *stage = nullptr,
                                                     bool u_ready = false, bool to_xt = false) {
  const int n = v.n, m = v.m, R = v.mr_cnt, ldS = v.ld;
  const int n8 = (n + 7) & ~7;
  const LRLayout lo = lr_layout(n, m, R, ldS);
  const double *dinv = v.lr, *Sinv = v.lr + lo.S;
  double *wc = v.lr + lo.wc, *ug = v.lr + lo.u;
  auto rho_i = [&](int i) -> double { return v.iseq[i] ? 1e3 * rho_bar : rho_bar; };
  auto body = [&](double *u, double *wr, bool zero_wr) __attribute__((always_inline)) {
    tm.sync();
    if (!u_ready) {
      for (int j = tm.tid; j < n; j += tm.nt) u[j] = dinv[j] * double(v.r[j]);
    } else if (u != ug) {
      for (int j = tm.tid; j < n; j += tm.nt) u[j] = ug[j];
    }
    if (zero_wr)
      for (int i = tm.tid; i < m; i += tm.nt) wr[i] = 0.0;
    tm.sync();
    // wc = B u over the multi-entry rows
    const Rows rm(tm, v.lm);
    stream_rows<double>(v.arp, v.aci, v.av, u, rm.g, rm.ng, R, rm.lane, rm.L,
                        [&](int r) __attribute__((always_inline)) { return v.mrows[r]; },
                        [&](int i) __attribute__((always_inline)) { return v.iseq[i]; },
                        [&](int r, int i, double a, unsigned char eq) __attribute__((always_inline)) {
                          if (rm.lane == 0) wc[r] = sqrt(eq ? 1e3 * rho_bar : rho_bar) * a;
                        });
    tm.sync();
    // w = S^-1 (B u), scattered to the rows of A with the factor R_m^1/2
    dense_rows_matvec(tm, Sinv, ldS, R, wc, [&](int r, double w) __attribute__((always_inline)) {
      const int i = v.mrows[r];
      wr[i] = sqrt(rho_i(i)) * w;
    });
    tm.sync();
    // K^-1 r = u - Delta^-1 B' w  (B' w through the rows of A'; zero on
    // single-entry rows)
    const Rows rn(tm, v.ln);
    rows_ahead(v.atrp, rn.g, rn.ng, n, [&](int j, int b, int e) __attribute__((always_inline)) {
      const double uj = u[j], dj = dinv[j];
      const double a = group_sum(seg_partial4<double>(v.atci, v.atv, b, e, rn.lane, rn.L, wr), rn.L);
      if (rn.lane == 0) {
        const double step = uj - dj * a;
        if (to_xt) v.xt[j] += step;
        else v.d[j] = T(step);
      }
    });
    tm.sync();
  };
  if (stage != nullptr && n8 + ((m + 7) & ~7) <= kStage) body(stage, stage + n8, true);
  else body(ug, v.lr + lo.wr, false);
}

// ------------------------------------------------------------------------
// One full solve of one QP (Algorithm 1 with the reduced-system PCG of
// Section 3.1), then the FP64 checks, statuses and unscaled outputs.
// ------------------------------------------------------------------------
template <class T, class Team>
__device__ __forceinline__ void solve_qp(const Team &tm, const QPView<T> &v, const DevSettings &set,
                         DenseLDS<T> *dl = nullptr, T *dB = nullptr, bool dense_ok = false,
                         DenseLDS<double> *dl64 = nullptr, double *G = nullptr, bool lr_ok = false,
                         double *stage = nullptr) {
  QPState &S = *v.st;
  const int n = v.n, m = v.m;
  const T sigma = T(set.sigma);
  const double c = S.c, cinv = 1.0 / c;
  double rho_bar = S.rho_bar;
  // rho_i in double for the iterate updates and residuals (the stored T copy
  // feeds only the PCG products)
  auto rho_of = [&](int i) -> double { return v.iseq[i] ? 1e3 * rho_bar : rho_bar; };
  const Rows rn(tm, v.ln), rm(tm, v.lm);
  const unsigned long long t_start = wall_clock64();
  unsigned long long ph = t_start, c_factor = 0, c_pcg = 0, c_update = 0, c_check = 0;
  auto lap = [&](unsigned long long &acc) {   // phase timer (team leader's clock)
    const unsigned long long t = wall_clock64();
    acc += t - ph;
    ph = t;
  };

  set_rho_and_precond(tm, v, rho_bar, set.sigma);
  // exact preconditioner of K (dense factor, or the low-rank Woodbury form):
  // the stored factor is reused while rho-bar is unchanged
  const int pre_kind = (v.dense == 1 && dense_ok) ? 1
                     : (v.dense == 2 && lr_ok) ? 2
                     : (v.dense == 3 && lr_ok) ? 3 : 0;
  auto refactor = [&]() __attribute__((always_inline)) -> bool {
    if constexpr (std::is_same<Team, WGTeam>::value) {
      if (pre_kind == 1) return form_and_factor<T>(tm, v, *dl, dB, set.sigma);
      if (pre_kind == 3) return band_form_and_factor<T>(tm, v, *dl64, G, set.sigma, rho_bar);
      return lowrank_form_and_factor<T>(tm, v, *dl64, G, set.sigma, rho_bar);
    } else {
      return false;
    }
  };
  auto apply_pre = [&]() __attribute__((always_inline)) {
    if constexpr (std::is_same<Team, WGTeam>::value) {
      if (pre_kind == 1) precondition_dense(tm, v, *dl);
      else precondition_lowrank(tm, v, rho_bar, stage);
    }
  };
  bool use_dense = false;
  if constexpr (std::is_same<Team, WGTeam>::value) {
    if (pre_kind != 0) {
      use_dense = true;
      if (S.factor_rho != rho_bar) {
        ph = wall_clock64();
        use_dense = refactor();
        if (tm.tid == 0) S.factor_rho = use_dense ? rho_bar : 0.0;
        tm.sync();
        lap(c_factor);
      }
    }
  }

  // initial iterate: continue, zeros, or the warm start of Section 6
  const int mode = S.init_mode;
  if (mode == 1) {
    for (int j = tm.tid; j < n; j += tm.nt) { v.x[j] = 0.0; v.xt[j] = 0.0; }
    for (int i = tm.tid; i < m; i += tm.nt) { v.z[i] = 0.0; v.y[i] = 0.0; }
  } else if (mode == 2) {
    for (int j = tm.tid; j < n; j += tm.nt) {
      const double xv = v.Dinv[j] * v.xws[j];
      v.x[j] = xv; v.xt[j] = xv;
    }
    for (int i = tm.tid; i < m; i += tm.nt) v.y[i] = c * v.Einv[i] * v.yws[i];
    tm.sync();
    for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
      const double a = group_sum(seg_partial4<double>(v.aci, v.av, b, e, lane, L, v.x), L);
      if (lane == 0) v.z[i] = a;
    });
  } else {
    for (int j = tm.tid; j < n; j += tm.nt) v.xt[j] = v.x[j];
  }
  tm.sync();
  // zt = A xt ; s = rho (z - zt) - y  (feeds the first right-hand side);
  // both in double from the double copy of A (a mixed-precision refinement:
  // each linear solve starts from a residual computed in FP64)
  for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
    const double a = group_sum(seg_partial4<double>(v.aci, v.av, b, e, lane, L, v.xt), L);
    if (lane == 0) {
      v.zt64[i] = a;
      if (sizeof(T) == 4) v.zt[i] = T(a);
      v.s64[i] = rho_of(i) * (v.z[i] - a) - v.y[i];
    }
  });
  tm.sync();

  int k = 0, status = 6 /* unsolved */, pcg_total = 0, rho_updates = 0;
  bool have_check = false;
  double prs = 0.0, drs = 0.0, pnorm = 0.0, dnorm = 0.0, bnorm = -1.0;
  double res_prim = 0.0, res_dual = 0.0, eps_prim = 0.0, eps_dual = 0.0;
  int bad = 0;
  const double floor_rel = sizeof(T) == 4 ? 1e-6 : 1e-12;
  auto pcg_tol = [&](double b0) -> double {
    return have_check ? fmax(set.pcg_tol_frac * fmin(prs, drs), floor_rel * fmax(dnorm, 1e-30))
                      : 1e-2 * set.pcg_tol_frac * b0;
  };
  // LDS staging of the vectors a pass gathers from (workgroup team): the
  // gathers then hit LDS and only the streamed matrix comes from memory
  const int n8 = (n + 7) & ~7, m8 = (m + 7) & ~7;
  const bool stg_start = stage != nullptr && m8 + n8 <= kStage;
  const bool stg_upd = stage != nullptr && n8 <= kStage;
  const bool stg_kp = stage != nullptr && (int64_t)(n8 + m8) * (int64_t)sizeof(T) <= 8LL * kStage;
  T *stT = reinterpret_cast<T *>(stage);

  // the low-rank form, the band factor and (FP64 path) the dense factor
  // solve K exactly in FP64: there the step is the direct one (Section 3.1
  // with the reduced matrix), x~ += K^-1 r, and no PCG runs.  The start pass
  // leaves u = Delta^-1 r (low-rank form) or r itself (band factor) in the
  // factor's block, in FP64; the dense factor solves from r in place.
  const int64_t lr_u = pre_kind == 2 ? lr_layout(n, m, v.mr_cnt, v.ld).u
                     : pre_kind == 3 ? band_layout(n, v.ld).r : 0;

  ph = wall_clock64();
  while (true) {
    // the exact factors in FP64 -- low-rank form, band factor, and the
    // dense factor of the FP64 path -- take the direct step; the FP32 dense
    // factor preconditions PCG
    const bool direct =
        (pre_kind == 2 || pre_kind == 3 || (pre_kind == 1 && sizeof(T) == 8)) && use_dense;
    // --- PCG start: r = b - K xt with b = sigma x - q + A'(rho z - y)
    //     (Section 3.1, indirect method), K = P + sigma I + A' R A, using
    //     A xt = zt:  r = sigma (x - xt) - q - P xt + A' s
    double red[2];
    red[0] = 0.0; red[1] = 0.0;
    auto start_pass = [&](const double *s_src, const double *x_src) __attribute__((always_inline)) {
      rows_ahead2(v.atrp, v.prp, rn.g, rn.ng, n,
                  [&](int j, int ab, int ae, int pb, int pe) __attribute__((always_inline)) {
        // the row's own values are loaded before the gathers (they do not
        // depend on them), so their latency overlaps
        const double xj = v.x[j], xtj = v.xt[j], qj = v.q64[j];
        double a = seg_partial4<double>(v.atci, v.atv, ab, ae, rn.lane, rn.L, s_src) -
                   seg_partial4<double>(v.pci, v.pv, pb, pe, rn.lane, rn.L, x_src);
        a = group_sum(a, rn.L);
        if (rn.lane == 0) {
          const double r64 = set.sigma * (xj - xtj) - qj + a;
          const T rj = T(r64);
          v.r[j] = rj;
          if (direct && pre_kind != 1) v.lr[lr_u + j] = pre_kind == 2 ? v.lr[j] * r64 : r64;
          red[1] = fmax(red[1], fabs(r64));
          if (!use_dense) {
            const T dj = v.minv[j] * rj;
            v.d[j] = dj; v.p[j] = dj;
            red[0] += double(rj * dj);
          }
        }
      });
    };
    if (stg_start) {
      for (int i = tm.tid; i < m; i += tm.nt) stage[i] = v.s64[i];
      for (int j = tm.tid; j < n; j += tm.nt) stage[m8 + j] = v.xt[j];
      tm.sync();
      start_pass(stage, stage + m8);
    } else {
      start_pass(v.s64, v.xt);
    }
    // the dense preconditioner is a factor of K itself: one PCG step with it
    // is the exact solve.  With an exact factor every ADMM step takes its
    // linear solve, as the direct method does (skipping it while the residual
    // is under the inner tolerance ends at another eps-solution)
    if constexpr (std::is_same<Team, WGTeam>::value) {
      if (use_dense) {
        tm.template reduce<0, 1>(red + 1);
        if (direct) {
          if (pre_kind == 3) {
            band_direct_step(tm, v, stage, dl64->ys);
          } else if (pre_kind == 1) {
            // FP64 dense factor: d = K^-1 r, x~ += d
            apply_pre();
            for (int j = tm.tid; j < n; j += tm.nt) v.xt[j] += double(v.d[j]);
            tm.sync();
          } else {
            precondition_lowrank(tm, v, rho_bar, stage, true, true);
          }
        } else {
          apply_pre();
          for (int j = tm.tid; j < n; j += tm.nt) {
            const T dj = v.d[j];
            v.p[j] = dj;
            red[0] += double(v.r[j] * dj);
          }
          tm.template reduce<1, 0>(red);
        }
      } else {
        tm.template reduce<1, 1>(red);
      }
    } else {
      tm.template reduce<1, 1>(red);
    }
    double rz = red[0], rinf = red[1];
    if (bnorm < 0.0) bnorm = rinf;
    // inner tolerance (reading): kappa * min(prim, dual residual) of the last
    // check, floored relative to the dual normaliser; 1e-2 kappa of the
    // first residual before the first check (kappa = pcg_tol_frac)
    const double tol = pcg_tol(bnorm);
    int it = direct ? 1 : 0;
    // with the exact factor the first step is taken even below the inner
    // tolerance (unless the residual is exactly zero)
    const bool forced0 = !(rinf > tol);
    while (!direct && (rinf > tol || (forced0 && it == 0 && rinf > 0.0)) &&
           it < set.pcg_max_iter) {
      // t = R A p ; w = P p + sigma p + A' t ; p'w
      auto kprod = [&](const T *p_src, T *t_dst, const T *t_src) __attribute__((always_inline)) {
        for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
          const T ri = v.rho[i];
          const T a = group_sum(seg_partial4<T>(v.aci, v.av, b, e, lane, L, p_src), L);
          if (lane == 0) t_dst[i] = ri * a;
        });
        tm.sync();
        red[0] = 0.0;
        rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n,
                    [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
          const T pj = v.p[j];
          T a = seg_partial4<T>(v.pci, v.pv, pb, pe, rn.lane, rn.L, p_src) +
                seg_partial4<T>(v.atci, v.atv, ab, ae, rn.lane, rn.L, t_src);
          a = group_sum(a, rn.L);
          if (rn.lane == 0) {
            const T wj = a + sigma * pj;
            v.w[j] = wj;
            red[0] += double(pj * wj);
          }
        });
      };
      if (stg_kp) {
        for (int j = tm.tid; j < n; j += tm.nt) stT[j] = v.p[j];
        tm.sync();
        kprod(stT, stT + n8, stT + n8);
      } else {
        kprod(v.p, v.t, v.t);
      }
      tm.template reduce<1, 0>(red);
      const double pw = red[0];
      if (!(pw > 0.0) || !isfinite(pw)) {
        // K is positive definite, so a curvature that is not positive comes
        // from rounding once the residual is small: after the first step, or
        // on a forced first step below the inner tolerance, x~ stays and the
        // inner solve ends; a non-positive curvature on a first step above
        // the tolerance, or a non-finite one, is a breakdown
        if ((it == 0 && !forced0) || !isfinite(pw)) bad |= 1;
        break;
      }
      const double a_d = rz / pw;
      const T a_step = T(a_d);
      red[0] = 0.0; red[1] = 0.0;
      for (int j = tm.tid; j < n; j += tm.nt) {
        v.xt[j] += a_d * double(v.p[j]);
        const T rj = v.r[j] - a_step * v.w[j];
        v.r[j] = rj;
        red[1] = fmax(red[1], fabs(double(rj)));
        if (!use_dense) {
          const T dj = v.minv[j] * rj;
          v.d[j] = dj;
          red[0] += double(rj * dj);
        }
      }
      bool converged = false;
      if constexpr (std::is_same<Team, WGTeam>::value) {
        if (use_dense) {
          tm.template reduce<0, 1>(red + 1);
          converged = red[1] <= tol;
          if (!converged) {
            apply_pre();
            for (int j = tm.tid; j < n; j += tm.nt) red[0] += double(v.r[j] * v.d[j]);
            tm.template reduce<1, 0>(red);
          }
        } else {
          tm.template reduce<1, 1>(red);
        }
      } else {
        tm.template reduce<1, 1>(red);
      }
      if (converged) { ++it; break; }
      const T beta = T(red[0] / rz);
      rz = red[0];
      rinf = red[1];
      for (int j = tm.tid; j < n; j += tm.nt) v.p[j] = v.d[j] + beta * v.p[j];
      tm.sync();
      ++it;
      if (!(rz > 0.0)) break;
    }
    pcg_total += it;
    lap(c_pcg);
    ++k;
    const bool do_check = (set.check_every > 0 && k % set.check_every == 0) || k >= set.max_iter;
    // --- Algorithm 1 updates: x relaxed; v = alpha zt + (1-alpha) z + y/rho;
    //     z = Pi(v); y = rho (v - z)  (v-form of Section 3.3)
    for (int j = tm.tid; j < n; j += tm.nt) {
      const double xtj = v.xt[j];
      const double xn = set.alpha * xtj + (1.0 - set.alpha) * v.x[j];
      if (do_check) v.dx[j] = xn - v.x[j];
      v.x[j] = xn;
      if (stg_upd) stage[j] = xtj;
    }
    if (stg_upd) tm.sync();
    auto upd_pass = [&](const double *xt_src) __attribute__((always_inline)) {
      for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
        const double zi = v.z[i], yi = v.y[i], ri = rho_of(i);
        const double a64 = group_sum(seg_partial4<double>(v.aci, v.av, b, e, lane, L, xt_src), L);
        if (lane == 0) {
          const double vv = set.alpha * a64 + (1.0 - set.alpha) * zi + yi / ri;
          const double zn = fmin(fmax(vv, v.l64[i]), v.u64[i]);
          const double yn = ri * (vv - zn);
          if (do_check) v.dy[i] = yn - yi;
          if (sizeof(T) == 4) v.zt[i] = T(a64);
          v.zt64[i] = a64;
          v.z[i] = zn;
          v.y[i] = yn;
          v.s64[i] = ri * (zn - a64) - yn;
        }
      });
    };
    if (stg_upd) upd_pass(stage);
    else upd_pass(v.xt);
    tm.sync();
    lap(c_update);
    if (!do_check) continue;

    // --- FP64 termination check (Sections 3.4, 5.1): unscaled residuals
    //     and tolerances, then the infeasibility tests on dy, dx.
    //  sums : [0] u'dy+ + l'dy-, [1] q'dx
    //  maxes: [2] |E^-1(Ax-z)| [3] |E^-1 Ax| [4] |E^-1 z| [5] |Ax-z| [6] |Ax| [7] |z|
    //         [8] |D^-1(Px+q+A'y)| [9] |D^-1 Px| [10] |D^-1 A'y| [11] |D^-1 q|
    //         [12] |Px+q+A'y| [13] |Px| [14] |A'y| [15] |q|
    //         [16] |E dy| [17] |D^-1 A'dy| [18] inf-bound hit
    //         [19] |D dx| [20] |D^-1 P dx| [21] both-finite |E^-1 A dx|
    //         [22] lower-only -(E^-1 A dx) [23] upper-only (E^-1 A dx) [24] elapsed s
    double chk[25];
#pragma unroll
    for (int kk = 0; kk < 25; ++kk) chk[kk] = 0.0;
    for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
      double ax = 0.0, adx = 0.0;
      for (int kq = b + lane; kq < e; kq += L) {
        const double a = v.a64[kq];
        const int cj = v.aci[kq];
        ax += a * double(v.x[cj]);
        adx += a * v.dx[cj];
      }
      ax = group_sum(ax, L);
      adx = group_sum(adx, L);
      if (lane == 0) {
        const double zi = double(v.z[i]), ei = v.Einv[i];
        chk[2] = fmax(chk[2], fabs(ei * (ax - zi)));
        chk[3] = fmax(chk[3], fabs(ei * ax));
        chk[4] = fmax(chk[4], fabs(ei * zi));
        chk[5] = fmax(chk[5], fabs(ax - zi));
        chk[6] = fmax(chk[6], fabs(ax));
        chk[7] = fmax(chk[7], fabs(zi));
        const double dyi = v.dy[i];
        chk[16] = fmax(chk[16], fabs(v.E[i] * dyi));
        // reading: only dy_i > 0 meets u_i and only dy_i < 0 meets l_i; an
        // infinite bound met this way fails the test
        // (flags are folded in with fmax/select, not by a conditional store
        // of a constant: hipcc's backend was seen to drop such stores into
        // a per-thread reduction array inside a divergent loop)
        const double bnd = dyi > 0.0 ? v.u64[i] : (dyi < 0.0 ? v.l64[i] : 0.0);
        const bool hit = isinf(bnd);
        chk[18] = fmax(chk[18], hit ? 1.0 : 0.0);
        chk[0] += hit ? 0.0 : bnd * dyi;
        const double wv = ei * adx;
        const bool lf = !isinf(v.l64[i]), uf = !isinf(v.u64[i]);
        chk[21] = fmax(chk[21], (lf && uf) ? fabs(wv) : 0.0);
        chk[22] = fmax(chk[22], (lf && !uf) ? -wv : 0.0);
        chk[23] = fmax(chk[23], (!lf && uf) ? wv : 0.0);
      }
    });
    for (int j = rn.g; j < n; j += rn.ng) {
      double px = 0.0, pdx = 0.0, aty = 0.0, atdy = 0.0;
      for (int kq = v.prp[j] + rn.lane; kq < v.prp[j + 1]; kq += rn.L) {
        const double a = v.p64[kq];
        const int cj = v.pci[kq];
        px += a * double(v.x[cj]);
        pdx += a * v.dx[cj];
      }
      for (int kq = v.atrp[j] + rn.lane; kq < v.atrp[j + 1]; kq += rn.L) {
        const double a = v.at64[kq];
        const int ci = v.atci[kq];
        aty += a * double(v.y[ci]);
        atdy += a * v.dy[ci];
      }
      px = group_sum(px, rn.L); pdx = group_sum(pdx, rn.L);
      aty = group_sum(aty, rn.L); atdy = group_sum(atdy, rn.L);
      if (rn.lane == 0) {
        const double qj = v.q64[j], di = v.Dinv[j];
        const double rd = px + qj + aty;
        chk[8] = fmax(chk[8], fabs(di * rd));
        chk[9] = fmax(chk[9], fabs(di * px));
        chk[10] = fmax(chk[10], fabs(di * aty));
        chk[11] = fmax(chk[11], fabs(di * qj));
        chk[12] = fmax(chk[12], fabs(rd));
        chk[13] = fmax(chk[13], fabs(px));
        chk[14] = fmax(chk[14], fabs(aty));
        chk[15] = fmax(chk[15], fabs(qj));
        chk[17] = fmax(chk[17], fabs(di * atdy));
        const double dxj = v.dx[j];
        chk[19] = fmax(chk[19], fabs(v.D[j] * dxj));
        chk[20] = fmax(chk[20], fabs(di * pdx));
        chk[1] += qj * dxj;
      }
    }
    if (tm.tid == 0) chk[24] = double(wall_clock64() - t_start) * set.wall_tick_s;
    tm.template reduce<2, 23>(chk);
    res_prim = chk[2];
    eps_prim = set.eps_abs + set.eps_rel * fmax(chk[3], chk[4]);
    res_dual = cinv * chk[8];
    eps_dual = set.eps_abs + set.eps_rel * cinv * fmax(chk[9], fmax(chk[10], chk[11]));
    prs = chk[5]; pnorm = fmax(chk[6], chk[7]);
    drs = chk[12]; dnorm = fmax(chk[13], fmax(chk[14], chk[15]));
    have_check = true;
    lap(c_check);
    // non-finite iterates: the maxima above drop NaN, the sums keep it; stop
    // as unsolved rather than read the dropped terms as converged
    if (!isfinite(chk[0]) || !isfinite(chk[1])) { bad |= 2; status = 6; break; }
    if (res_prim <= eps_prim && res_dual <= eps_dual) { status = 1; break; }
    // primal infeasibility (Section 5.1, strict-sign reading)
    {
      const double ndy = chk[16];
      if (ndy > 0.0 && chk[18] == 0.0 && chk[0] < -set.eps_pinf * ndy &&
          chk[17] <= set.eps_pinf * ndy) { status = 2; break; }
    }
    // dual infeasibility (Section 5.1)
    {
      const double ndx = chk[19], tl = set.eps_dinf * ndx;
      if (ndx > 0.0 && chk[1] < -c * tl && chk[20] <= c * tl && chk[21] <= tl &&
          chk[22] <= tl && chk[23] <= tl) { status = 3; break; }
    }
    if (set.time_limit > 0.0 && chk[24] >= set.time_limit) { status = 5; break; }
    if (k >= set.max_iter) { status = 4; break; }
    if (bad) { status = 6; break; }
    // rho-bar rule (Section 5.2), scaled quantities; readings: skip on zero
    // normalisers, clamp to [1e-6, 1e6], apply when at least 5x larger or
    // smaller
    if (set.adaptive_rho && pnorm > 0.0 && dnorm > 0.0 && drs > 0.0) {
      double rnew = rho_bar * sqrt((prs / pnorm) / (drs / dnorm));
      rnew = fmin(fmax(rnew, 1e-6), 1e6);
      if (rnew >= 5.0 * rho_bar || rnew <= rho_bar / 5.0) {
        rho_bar = rnew;
        ++rho_updates;
        set_rho_and_precond(tm, v, rho_bar, set.sigma);
        if constexpr (std::is_same<Team, WGTeam>::value) {
          if (pre_kind != 0) {
            use_dense = refactor();
            if (tm.tid == 0) S.factor_rho = use_dense ? rho_bar : 0.0;
            tm.sync();
            lap(c_factor);
          }
        }
        for (int i = tm.tid; i < m; i += tm.nt)
          v.s64[i] = rho_of(i) * (v.z[i] - v.zt64[i]) - v.y[i];
        tm.sync();
      }
    }
  }

  // --- unscale (Section 5.1) and objective on the scaled data divided by c
  double red[1];
  red[0] = 0.0;
  for (int j = rn.g; j < n; j += rn.ng) {
    double px = 0.0;
    for (int kq = v.prp[j] + rn.lane; kq < v.prp[j + 1]; kq += rn.L)
      px += v.p64[kq] * double(v.x[v.pci[kq]]);
    px = group_sum(px, rn.L);
    if (rn.lane == 0) {
      const double xj = double(v.x[j]);
      red[0] += 0.5 * xj * px + v.q64[j] * xj;
      v.xo[j] = v.D[j] * (status == 3 ? v.dx[j] : xj);
    }
  }
  for (int i = tm.tid; i < m; i += tm.nt) {
    v.yo[i] = cinv * v.E[i] * (status == 2 ? v.dy[i] : double(v.y[i]));
    v.zo[i] = v.Einv[i] * double(v.z[i]);
  }
  tm.template reduce<1, 0>(red);
  if (tm.tid == 0) {
    S.status = status;
    S.iter = k;
    S.pcg_iter = pcg_total;
    S.rho_updates = rho_updates;
    S.rho_bar = rho_bar;
    S.prim_res = res_prim; S.dual_res = res_dual;
    S.eps_prim = eps_prim; S.eps_dual = eps_dual;
    S.prs = prs; S.drs = drs; S.pnorm = pnorm; S.dnorm = dnorm;
    S.obj = status == 2 ? INFINITY : (status == 3 ? -INFINITY : cinv * red[0]);
    S.polish_status = 0;
    S.init_mode = 0;
    S.bad = bad;
    const double tk = set.wall_tick_s * 1e3;
    S.solve_ms = double(wall_clock64() - t_start) * tk;
    S.t_factor_ms = double(c_factor) * tk;
    S.t_pcg_ms = double(c_pcg) * tk;
    S.t_update_ms = double(c_update) * tk;
    S.t_check_ms = double(c_check) * tk;
  }
  tm.sync();
}

}  // namespace osqpmi
