// FP64 solution polishing (Section 4) on the device, one QP per workgroup.
//
// Active sets from the scaled dual iterate: L = {y_i < 0}, U = {y_i > 0}.
// The regularised reduced KKT system (eq. kkt_polish_reg)
//     [ P + dI   A_a' ] [x  ]   [ -q  ]
//     [ A_a     -dI   ] [y_a] = [ b_a ],  b_a = l_L, u_U
// is solved through its condensed SPD form
//     M x = -q + A_a' b_a / d,   M = P + dI + A_a'A_a / d,   y_a = (A_a x - b_a) / d.
// Single-entry active rows only add to the diagonal of M; the active rows
// with several entries form B = A_m / sqrt(d).  M is either formed densely
// and factored by a dense Cholesky, or -- when P is diagonal and the
// multi-entry rows are few (flag plr of the QP) -- kept as Delta + B'B and
// solved by the Woodbury identity with the small capacitance matrix
// S = I + B Delta^-1 B'.  Then the fixed number of iterative-refinement
// passes of eq. iterative_refinement against the unregularised matrix (eq.
// kkt_polish), each one more solve with M.  The polished point is accepted
// when its unscaled residuals do not exceed the ADMM ones and the duals of
// the active inequality rows keep their signs (reading; an equality row's
// dual may take either sign); otherwise the ADMM solution stays.
#pragma once

#include "dense.h"
#include "solver_device.h"

namespace osqpmi {

constexpr int kMaxPolishWaves = 16;   // polishing workgroups have at most 1024 threads

// Workspace (doubles) of one polishing slot.  Dense: M (n x ldm), the
// inverses of its 64 x 64 diagonal blocks, B (rmax x n).  Low-rank: Delta^-1,
// u, S (rmax x ldS), its block inverses, w compact, w by row, G (rmax x ldg).
// Then the vectors of both variants.
__host__ __device__ inline int64_t polish_ws_doubles(int n, int m, int rmax, bool lowrank) {
  const int64_t n8 = (n + 7) & ~7, m8 = (m + 7) & ~7, r8 = (rmax + 7) & ~7;
  int64_t head;
  if (lowrank)
    head = 2 * n8 + (int64_t)rmax * r8 + (int64_t)((rmax + 63) / 64) * 4096 + r8 + m8 +
           (int64_t)rmax * n8;
  else
    head = n * n8 + (int64_t)((n + 63) / 64) * 4096 + (int64_t)rmax * n;
  return ((head + 7) & ~int64_t(7)) + 3 * n8 + 5 * m8 + 64;
}

template <class T>
__device__ __forceinline__ void polish_qp(const WGTeam &tm, DenseLDS<double> &s, const QPView<T> &v,
                                          const DevSettings &set, double *ws, int rmax, bool lowrank) {
  const int n = v.n, m = v.m;
  const double delta = set.delta, dinv_d = 1.0 / delta, rs = sqrt(dinv_d);
  const double c = v.st->c, cinv = 1.0 / c;
  const unsigned long long t0 = wall_clock64();
  const int n8 = (n + 7) & ~7, m8 = (m + 7) & ~7, r8 = (rmax + 7) & ~7;
  const int nblk = (n + kSB - 1) / kSB, rblk = (rmax + kSB - 1) / kSB;
  // matrix part
  double *M = ws, *Minv = nullptr, *B = nullptr;                 // dense
  double *Dl = ws, *u = nullptr, *S = nullptr, *Sinv = nullptr;  // low-rank
  double *wc = nullptr, *wr = nullptr, *G = nullptr;
  int64_t head;
  if (lowrank) {
    u = Dl + n8;
    S = u + n8;
    Sinv = S + (size_t)rmax * r8;
    wc = Sinv + (size_t)rblk * 4096;
    wr = wc + r8;
    G = wr + m8;
    head = (G - ws) + (int64_t)rmax * n8;
  } else {
    Minv = M + (size_t)n * n8;
    B = Minv + (size_t)nblk * 4096;
    head = (B - ws) + (int64_t)rmax * n;
  }
  double *act = ws + ((head + 7) & ~int64_t(7));   // m: -1, 0, +1
  double *bact = act + m8;                         // m
  double *tx = bact + m8, *ty = tx + n8;           // n, m
  double *rx = ty + m8, *ry = rx + n8;             // n, m
  double *g = ry + m8;                             // n
  int *multi = reinterpret_cast<int *>(g + n8);    // m
  __shared__ int R_sh;

  for (int i = tm.tid; i < m; i += tm.nt) {
    const double yi = double(v.y[i]);
    const double a = yi < 0.0 ? -1.0 : (yi > 0.0 ? 1.0 : 0.0);
    act[i] = a;
    bact[i] = a < 0.0 ? v.l64[i] : (a > 0.0 ? v.u64[i] : 0.0);
  }
  tm.sync();
  // active multi-entry rows, in row order: a ballot per wave, the waves'
  // counts in LDS, then each thread's position (deterministic)
  __shared__ int wcount[kMaxPolishWaves];
  // the reset is ordered before every read of the count, also when the QP
  // has no multi-entry rows and the loop below never runs (R_sh still holds
  // the previous QP's count in this workgroup's LDS)
  if (tm.tid == 0) R_sh = 0;
  tm.sync();
  {
    const int lane = tm.tid & (kWave - 1), wv = tm.tid >> 6, nw = tm.nt >> 6;
    for (int r0 = 0; r0 < v.mr_cnt; r0 += tm.nt) {
      const int r = r0 + tm.tid;
      const int i = r < v.mr_cnt ? v.mrows[r] : 0;
      const bool f = r < v.mr_cnt && act[i] != 0.0;
      const unsigned long long bal = __ballot(f);
      const int below = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[wv] = __popcll(bal);
      tm.sync();
      int off = R_sh;
      for (int w = 0; w < wv; ++w) off += wcount[w];
      if (f) multi[off + below] = i;
      tm.sync();
      if (tm.tid == 0) {
        int t = R_sh;
        for (int w = 0; w < nw; ++w) t += wcount[w];
        R_sh = t;
      }
      tm.sync();
    }
  }
  const int R = min(R_sh, rmax);
  const Rows rn(tm, v.ln), rm(tm, v.lm);
  bool ok_fact;
  if (lowrank) {
    // Delta = diag(P) + d + single-entry active rows a^2 / d;  G = B Delta^-1/2
    // ry (free until the refinement) marks the single-entry active rows
    for (int i = tm.tid; i < m; i += tm.nt)
      ry[i] = (act[i] != 0.0 && v.arp[i + 1] - v.arp[i] == 1) ? 1.0 : 0.0;
    for (size_t e = tm.tid; e < (size_t)R * n8; e += tm.nt) G[e] = 0.0;
    for (int i = tm.tid; i < m; i += tm.nt) wr[i] = 0.0;
    tm.sync();
    rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n,
                [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
      double a = 0.0;
      for (int k = pb + rn.lane; k < pe; k += rn.L)
        if (v.pci[k] == j) a += v.p64[k];
      a += seg_sum4<double>(v.atci, v.at64, ab, ae, rn.lane, rn.L,
                            [&](double e, int i) __attribute__((always_inline)) {
                              return ry[i] * e * e * dinv_d;
                            });
      a = group_sum(a, rn.L);
      if (rn.lane == 0) Dl[j] = 1.0 / (delta + a);
    });
    tm.sync();
    for (int r = rm.g; r < R; r += rm.ng) {
      const int i = multi[r];
      seg_each4(v.aci, v.a64, v.arp[i], v.arp[i + 1], rm.lane, rm.L,
                [&](int j, double a) __attribute__((always_inline)) {
                  G[(size_t)r * n8 + j] = a * rs * sqrt(Dl[j]);
                });
    }
    tm.sync();
    dense_gram_lower(tm, s, G, n8, R, n, S, r8);
    for (int r = tm.tid; r < R; r += tm.nt) S[(size_t)r * r8 + r] += 1.0;
    tm.sync();
    ok_fact = dense_cholesky<double>(tm, s, S, r8, R) && R_sh <= rmax;
    if (ok_fact) dense_invert_diag<double>(tm, s, S, r8, R, Sinv);
  } else {
    for (size_t e = tm.tid; e < (size_t)n * n8; e += tm.nt) M[e] = 0.0;
    for (size_t e = tm.tid; e < (size_t)R * n; e += tm.nt) B[e] = 0.0;
    tm.sync();
    // P + d I, plus the single-entry active rows on the diagonal
    for (int j = tm.tid; j < n; j += tm.nt) {
      for (int k = v.prp[j]; k < v.prp[j + 1]; ++k) M[(size_t)j * n8 + v.pci[k]] = v.p64[k];
      double dsum = delta;
      for (int k = v.atrp[j]; k < v.atrp[j + 1]; ++k) {
        const int i = v.atci[k];
        if (act[i] != 0.0 && v.arp[i + 1] - v.arp[i] == 1) dsum += v.at64[k] * v.at64[k] * dinv_d;
      }
      M[(size_t)j * n8 + j] += dsum;
    }
    for (int r = tm.tid; r < R; r += tm.nt) {
      const int i = multi[r];
      for (int k = v.arp[i]; k < v.arp[i + 1]; ++k) B[(size_t)r * n + v.aci[k]] = v.a64[k];
    }
    tm.sync();
    dense_syrk_tn<double>(tm, s, M, n8, B, n, R, n, dinv_d);
    ok_fact = dense_cholesky<double>(tm, s, M, n8, n) && R_sh <= rmax;
    if (ok_fact) dense_invert_diag<double>(tm, s, M, n8, n, Minv);
  }
  if (!ok_fact) {
    if (tm.tid == 0) v.st->polish_status = -1;
    tm.sync();
    return;
  }
  // g <- M^-1 g (in place)
  auto msolve = [&]() __attribute__((always_inline)) {
    if (lowrank) {
      for (int j = tm.tid; j < n; j += tm.nt) u[j] = Dl[j] * g[j];
      tm.sync();
      stream_rows<double>(v.arp, v.aci, v.a64, u, rm.g, rm.ng, R, rm.lane, rm.L,
                          [&](int r) __attribute__((always_inline)) { return multi[r]; },
                          [&](int) __attribute__((always_inline)) { return 0; },
                          [&](int r, int, double a, int) __attribute__((always_inline)) {
                            if (rm.lane == 0) wc[r] = rs * a;
                          });
      tm.sync();
      dense_solve_llt<double>(tm, s, S, r8, R, Sinv, wc);
      for (int r = tm.tid; r < R; r += tm.nt) wr[multi[r]] = rs * wc[r];
      tm.sync();
      rows_ahead(v.atrp, rn.g, rn.ng, n, [&](int j, int b, int e) __attribute__((always_inline)) {
        const double uj = u[j], dj = Dl[j];
        const double a = group_sum(seg_partial4<double>(v.atci, v.at64, b, e, rn.lane, rn.L, wr), rn.L);
        if (rn.lane == 0) g[j] = uj - dj * a;
      });
      tm.sync();
    } else {
      dense_solve_llt<double>(tm, s, M, n8, n, Minv, g);
    }
  };
  // first solve: rhs = -q + A_a' b_a / d
  // (bact is 0 on inactive rows)
  rows_ahead(v.atrp, rn.g, rn.ng, n, [&](int j, int b, int e) __attribute__((always_inline)) {
    const double qj = v.q64[j];
    const double a = group_sum(seg_partial4<double>(v.atci, v.at64, b, e, rn.lane, rn.L, bact), rn.L);
    if (rn.lane == 0) g[j] = -qj + a * dinv_d;
  });
  tm.sync();
  msolve();
  for (int j = tm.tid; j < n; j += tm.nt) tx[j] = g[j];
  tm.sync();
  for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
    const double ai = act[i], bi = bact[i];
    const double a = group_sum(seg_partial4<double>(v.aci, v.a64, b, e, lane, L, tx), L);
    if (lane == 0) ty[i] = ai != 0.0 ? (a - bi) * dinv_d : 0.0;
  });
  tm.sync();
  // iterative refinement: t += (K + dK)^-1 (g - K t), K without d
  for (int it = 0; it < set.refine; ++it) {
    for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
      const double ai = act[i], bi = bact[i];
      const double a = group_sum(seg_partial4<double>(v.aci, v.a64, b, e, lane, L, tx), L);
      if (lane == 0) ry[i] = ai != 0.0 ? bi - a : 0.0;
    });
    tm.sync();
    // g = (-q - P t_x - A' t_y) + A' r_y / d: one pass over the rows of A'
    // gathers both t_y and r_y
    rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n,
                [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
      const double qj = v.q64[j];
      const double2 at = seg_partial4x2(v.atci, v.at64, ab, ae, rn.lane, rn.L, ty, ry);
      const double a = group_sum(seg_partial4<double>(v.pci, v.p64, pb, pe, rn.lane, rn.L, tx) + at.x,
                                 rn.L);
      const double ar = group_sum(at.y, rn.L);
      if (rn.lane == 0) g[j] = (-qj - a) + ar * dinv_d;
    });
    tm.sync();
    msolve();
    for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
      const double ai = act[i], ri = ry[i];
      const double a = group_sum(seg_partial4<double>(v.aci, v.a64, b, e, lane, L, g), L);
      if (lane == 0 && ai != 0.0) ty[i] += (a - ri) * dinv_d;
    });
    tm.sync();
    for (int j = tm.tid; j < n; j += tm.nt) tx[j] += g[j];
    tm.sync();
  }
  // residuals of the polished point (unscaled), z = Pi(A x)
  double red[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) red[k] = 0.0;
  for_a_rows(tm, v, rm, [&](int i, int b, int e, int lane, int L) __attribute__((always_inline)) {
    const double lo = v.l64[i], hi = v.u64[i], ei = v.Einv[i], ai = act[i], tyi = ty[i];
    const double ax = group_sum(seg_partial4<double>(v.aci, v.a64, b, e, lane, L, tx), L);
    if (lane == 0) {
      const double z = fmin(fmax(ax, lo), hi);
      ry[i] = z;   // keep z
      red[1] = fmax(red[1], fabs(ei * (ax - z)));
      red[2] = fmax(red[2], fabs(ei * ax));
      red[3] = fmax(red[3], fabs(ei * z));
      // sign flag folded in with fmax (a conditional store of the constant
      // was dropped by hipcc's backend in this loop); a row with l_i = u_i
      // has both bounds active, so its dual may take either sign
      const bool flip = !v.iseq[i] && ((ai < 0.0 && tyi > 0.0) || (ai > 0.0 && tyi < 0.0));
      red[8] = fmax(red[8], flip ? 1.0 : 0.0);
    }
  });
  rows_ahead2(v.prp, v.atrp, rn.g, rn.ng, n,
              [&](int j, int pb, int pe, int ab, int ae) __attribute__((always_inline)) {
    const double d = v.Dinv[j], q = v.q64[j], txj = tx[j];
    const double px = group_sum(seg_partial4<double>(v.pci, v.p64, pb, pe, rn.lane, rn.L, tx), rn.L);
    const double aty = group_sum(seg_partial4<double>(v.atci, v.at64, ab, ae, rn.lane, rn.L, ty), rn.L);
    if (rn.lane == 0) {
      red[0] += 0.5 * txj * px + q * txj;
      red[4] = fmax(red[4], fabs(d * (px + q + aty)));
      red[5] = fmax(red[5], fabs(d * px));
      red[6] = fmax(red[6], fabs(d * aty));
      red[7] = fmax(red[7], fabs(d * q));
    }
  });
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
    QPState &St = *v.st;
    St.polish_status = accept ? 1 : -1;
    if (accept) {
      St.obj = cinv * red[0];
      St.prim_res = prim;
      St.dual_res = dual;
      St.eps_prim = set.eps_abs + set.eps_rel * fmax(red[2], red[3]);
      St.eps_dual = set.eps_abs + set.eps_rel * cinv * fmax(red[5], fmax(red[6], red[7]));
    }
    St.polish_ms = double(wall_clock64() - t0) * set.wall_tick_s * 1e3;
  }
  tm.sync();
}

}  // namespace osqpmi
