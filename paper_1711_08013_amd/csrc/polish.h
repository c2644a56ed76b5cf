// FP64 solution polishing (Section 4) on the device, one QP per workgroup.
//
// Active sets from the scaled dual iterate: L = {y_i < 0}, U = {y_i > 0}.
// The regularised reduced KKT system (eq. kkt_polish_reg)
//     [ P + dI   A_a' ] [x  ]   [ -q  ]
//     [ A_a     -dI   ] [y_a] = [ b_a ],  b_a = l_L, u_U
// is solved through its condensed SPD form
//     (P + dI + A_a'A_a / d) x = -q + A_a' b_a / d,   y_a = (A_a x - b_a) / d,
// formed densely (single-entry active rows only add to the diagonal, the
// others go through a rank-k update) and factored once by a dense Cholesky.
// Then the fixed number of iterative-refinement passes of eq.
// iterative_refinement against the unregularised matrix (eq. kkt_polish),
// each a pair of triangular solves.  The polished point is accepted when its
// unscaled residuals do not exceed the ADMM ones and the active duals keep
// their signs (reading); otherwise the ADMM solution stays.
#pragma once

#include "dense.h"
#include "solver_device.h"

namespace osqpmi {

struct PolishWS {
  double *base;
  long long stride;   // doubles per workgroup slot
  int nmax, rmax, mmax;
};

template <class T>
__device__ __forceinline__ void polish_qp(const WGTeam &tm, DenseLDS<double> &s, const QPView<T> &v,
                          const DevSettings &set, double *ws, int rmax) {
  const int n = v.n, m = v.m;
  const double delta = set.delta, dinv = 1.0 / delta;
  const double c = v.st->c, cinv = 1.0 / c;
  const unsigned long long t0 = wall_clock64();
  const int ldm = (n + 7) & ~7;                    // row stride of M (16-byte rows)
  const int nblk = (n + kSB - 1) / kSB;
  double *M = ws;                                  // n x ldm
  double *Minv = M + (size_t)n * ldm;              // nblk inverted 64 x 64 diagonal blocks
  double *B = Minv + (size_t)nblk * kSB * kSB;     // rmax x n
  double *act = B + (size_t)rmax * n;              // m: -1, 0, +1
  double *bact = act + m;                          // m
  double *tx = bact + m, *ty = tx + n;             // n, m
  double *rx = ty + m, *ry = rx + n;               // n, m
  double *g = ry + m;                              // n
  int *multi = reinterpret_cast<int *>(g + n);     // m
  __shared__ int R_sh;

  for (int i = tm.tid; i < m; i += tm.nt) {
    const double yi = double(v.y[i]);
    const double a = yi < 0.0 ? -1.0 : (yi > 0.0 ? 1.0 : 0.0);
    act[i] = a;
    bact[i] = a < 0.0 ? v.l64[i] : (a > 0.0 ? v.u64[i] : 0.0);
  }
  tm.sync();
  if (tm.tid == 0) {
    int R = 0;
    for (int i = 0; i < m; ++i)
      if (act[i] != 0.0 && v.arp[i + 1] - v.arp[i] >= 2) multi[R++] = i;
    R_sh = R;
  }
  for (size_t e = tm.tid; e < (size_t)n * ldm; e += tm.nt) M[e] = 0.0;
  tm.sync();
  const int R = min(R_sh, rmax);
  for (size_t e = tm.tid; e < (size_t)R * n; e += tm.nt) B[e] = 0.0;
  tm.sync();
  // P + d I, plus the single-entry active rows on the diagonal
  for (int j = tm.tid; j < n; j += tm.nt) {
    for (int k = v.prp[j]; k < v.prp[j + 1]; ++k) M[(size_t)j * ldm + v.pci[k]] = v.p64[k];
    double dsum = delta;
    for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) {
      const int i = v.atci[k];
      if (act[i] != 0.0 && v.arp[i + 1] - v.arp[i] == 1) dsum += v.at64[k] * v.at64[k] * dinv;
    }
    M[(size_t)j * ldm + j] += dsum;
  }
  for (int r = tm.tid; r < R; r += tm.nt) {
    const int i = multi[r];
    for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) B[(size_t)r * n + v.aci[k]] = v.a64[k];
  }
  tm.sync();
  dense_syrk_tn<double>(tm, s, M, ldm, B, n, R, n, dinv);
  const bool ok_fact = dense_cholesky<double>(tm, s, M, ldm, n) && R_sh <= rmax;
  if (ok_fact) dense_invert_diag<double>(tm, s, M, ldm, n, Minv);
  if (!ok_fact) {
    if (tm.tid == 0) v.st->polish_status = -1;
    tm.sync();
    return;
  }
  // first solve: rhs = -q + A_a' b_a / d
  for (int j = tm.tid; j < n; j += tm.nt) {
    double a = 0.0;
    for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) {
      const int i = v.atci[k];
      a += v.at64[k] * bact[i];     // bact is 0 on inactive rows
    }
    g[j] = -v.q64[j] + a * dinv;
  }
  tm.sync();
  dense_solve_llt<double>(tm, s, M, ldm, n, Minv, g);
  for (int j = tm.tid; j < n; j += tm.nt) tx[j] = g[j];
  tm.sync();
  for (int i = tm.tid; i < m; i += tm.nt) {
    double a = 0.0;
    if (act[i] != 0.0)
      for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) a += v.a64[k] * tx[v.aci[k]];
    ty[i] = act[i] != 0.0 ? (a - bact[i]) * dinv : 0.0;
  }
  tm.sync();
  // iterative refinement: t += (K + dK)^-1 (g - K t), K without d
  for (int it = 0; it < set.refine; ++it) {
    for (int i = tm.tid; i < m; i += tm.nt) {
      double a = 0.0;
      if (act[i] != 0.0)
        for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) a += v.a64[k] * tx[v.aci[k]];
      ry[i] = act[i] != 0.0 ? bact[i] - a : 0.0;
    }
    for (int j = tm.tid; j < n; j += tm.nt) {
      double a = 0.0;
      for (int k = v.prp[j]; k < v.prp[j + 1]; ++k) a += v.p64[k] * tx[v.pci[k]];
      for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) a += v.at64[k] * ty[v.atci[k]];
      rx[j] = -v.q64[j] - a;
    }
    tm.sync();
    for (int j = tm.tid; j < n; j += tm.nt) {
      double a = 0.0;
      for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) a += v.at64[k] * ry[v.atci[k]];
      g[j] = rx[j] + a * dinv;
    }
    tm.sync();
    dense_solve_llt<double>(tm, s, M, ldm, n, Minv, g);
    for (int i = tm.tid; i < m; i += tm.nt) {
      double a = 0.0;
      if (act[i] != 0.0)
        for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) a += v.a64[k] * g[v.aci[k]];
      if (act[i] != 0.0) ty[i] += (a - ry[i]) * dinv;
    }
    tm.sync();
    for (int j = tm.tid; j < n; j += tm.nt) tx[j] += g[j];
    tm.sync();
  }
  // residuals of the polished point (unscaled), z = Pi(A x)
  double red[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) red[k] = 0.0;
  for (int i = tm.tid; i < m; i += tm.nt) {
    double ax = 0.0;
    for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) ax += v.a64[k] * tx[v.aci[k]];
    const double z = fmin(fmax(ax, v.l64[i]), v.u64[i]);
    ry[i] = z;   // keep z
    const double e = v.Einv[i];
    red[1] = fmax(red[1], fabs(e * (ax - z)));
    red[2] = fmax(red[2], fabs(e * ax));
    red[3] = fmax(red[3], fabs(e * z));
    // sign flag folded in with fmax (a conditional store of the constant
    // was dropped by hipcc's backend in this loop)
    const bool flip = (act[i] < 0.0 && ty[i] > 0.0) || (act[i] > 0.0 && ty[i] < 0.0);
    red[8] = fmax(red[8], flip ? 1.0 : 0.0);
  }
  for (int j = tm.tid; j < n; j += tm.nt) {
    double px = 0.0, aty = 0.0;
    for (int k = v.prp[j]; k < v.prp[j + 1]; ++k) px += v.p64[k] * tx[v.pci[k]];
    for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) aty += v.at64[k] * ty[v.atci[k]];
    const double d = v.Dinv[j], q = v.q64[j];
    red[0] += 0.5 * tx[j] * px + q * tx[j];
    red[4] = fmax(red[4], fabs(d * (px + q + aty)));
    red[5] = fmax(red[5], fabs(d * px));
    red[6] = fmax(red[6], fabs(d * aty));
    red[7] = fmax(red[7], fabs(d * q));
  }
  tm.template reduce<1, 8>(red);
  const double prim = red[1], dual = cinv * red[4];
  const bool finite = isfinite(prim) && isfinite(dual) && isfinite(red[0]);
  const bool accept = finite && red[8] == 0.0 && prim <= v.st->prim_res && dual <= v.st->dual_res;
  if (accept) {
    for (int j = tm.tid; j < n; j += tm.nt) {
      v.xo[j] = v.D[j] * tx[j];
      v.x[j] = tx[j];
    }
    for (int i = tm.tid; i < m; i += tm.nt) {
      v.yo[i] = cinv * v.E[i] * ty[i];
      v.zo[i] = v.Einv[i] * ry[i];
      v.y[i] = ty[i];
      v.z[i] = ry[i];
    }
  }
  if (tm.tid == 0) {
    QPState &S = *v.st;
    S.polish_status = accept ? 1 : -1;
    if (accept) {
      S.obj = cinv * red[0];
      S.prim_res = prim;
      S.dual_res = dual;
      S.eps_prim = set.eps_abs + set.eps_rel * fmax(red[2], red[3]);
      S.eps_dual = set.eps_abs + set.eps_rel * cinv * fmax(red[5], fmax(red[6], red[7]));
    }
    S.polish_ms = double(wall_clock64() - t0) * set.wall_tick_s * 1e3;
  }
  tm.sync();
}

}  // namespace osqpmi
