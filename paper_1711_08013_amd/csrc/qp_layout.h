// Internal layout shared by the host setup code and the HIP kernels of
// osqp_mi.  A batch of QPs is packed block-diagonally: every n-sized vector
// of QP k lives at [xo, xo+n) of one concatenated array, every m-sized
// vector at [yo, yo+m); every sparse matrix is CSR with per-QP local row
// pointers (entries of QP k start at its *_nz base) and local column indices.
#pragma once

#include <cstdint>

namespace osqpmi {

// Per-QP descriptor (read-only on the device).
struct QPDesc {
  int n, m;
  int64_t xo, yo;            // vector offsets
  int64_t a_rp, at_rp, p_rp; // row-pointer array offsets (m+1, n+1, n+1 entries)
  int64_t a_nz, at_nz, p_nz; // entry offsets
  int lm, ln;                // lanes per row for passes over A rows / over P+A' rows
  int dense;                 // exact PCG preconditioner of P + sigma I + A'RA:
                             // 0 none (Jacobi), 1 dense Cholesky factor,
                             // 2 diagonal plus low rank (P diagonal; Woodbury),
                             // 3 block-tridiagonal factor after a bandwidth-
                             //   reducing ordering (band)
  int dld;                   // leading dimension of the dense factor / of S;
                             // the block size nb of the band factor
  int64_t dense_off;         // offset in the dense arena (1) or the FP64 low-rank
                             // arena (2, and 3: the band tiles live there too)
  int64_t mr_off;            // offset of the list of A rows with >= 2 entries
  int mr_cnt;                // length of that list
  int plr;                   // 1: polish through the low-rank (Woodbury) condensed solve
};

// Offsets (doubles) inside one QP's low-rank block: Delta^-1 at 0, then u
// (n), the capacitance matrix S (R x ldS; formed and factored there, then
// replaced by the full symmetric S^-1), w compact (R) and w scattered by row
// of A (m).  Every part starts on a multiple of 8 doubles.
struct LRLayout {
  int64_t u, S, wc, wr, total;
};
__host__ __device__ inline LRLayout lr_layout(int n, int m, int R, int ldS) {
  const int64_t n8 = (n + 7) & ~7, m8 = (m + 7) & ~7, R8 = (R + 7) & ~7;
  LRLayout L;
  L.u = n8;
  L.S = L.u + n8;
  L.wc = L.S + (int64_t)R * ldS;
  L.wr = L.wc + R8;
  L.total = L.wr + m8;
  return L;
}

// Band block of one QP (dense == 3, doubles, in the low-rank arena): block
// rows i = 0 .. ceil(n / nb) - 1 of the factor, each two nb x nb row-major
// tiles, Linv_i = L_ii^-1 (lower) at 2 i nb^2 and C_i = B_i L_ii^-T (upper
// triangular; zero for the last block row) at (2 i + 1) nb^2; then the FP64
// residual r (n, variable order) the direct step solves with.
struct BandLayout {
  int64_t tiles, r, total;
};
__host__ __device__ inline BandLayout band_layout(int n, int nb) {
  BandLayout L;
  L.tiles = 0;
  L.r = 2 * (int64_t)((n + nb - 1) / nb) * nb * nb;
  L.total = L.r + ((n + 7) & ~7);
  return L;
}
// Per-workgroup scratch (doubles) while a band factor is formed: kBandCopies
// copies of a block row's strip of K (nb x 2 nb: the sub-diagonal block
// beside the diagonal block), then D (nb x nb), Bp (nb x nb) and a 64 x 64
// tile for the inverse of the diagonal factor.
constexpr int kBandCopies = 4;
struct BandScratch {
  int64_t strip, D, Bp, X, total;
};
__host__ __device__ inline BandScratch band_scratch_layout(int nb) {
  BandScratch s;
  s.strip = 0;
  s.D = (int64_t)kBandCopies * 2 * nb * nb;
  s.Bp = s.D + (int64_t)nb * nb;
  s.X = s.Bp + (int64_t)nb * nb;
  s.total = s.X + 64 * 64;
  return s;
}
__host__ __device__ inline int64_t band_scratch(int nb) { return band_scratch_layout(nb).total; }

// Per-QP mutable state (device).
struct QPState {
  double c;             // cost scaling (Section 5.1)
  double rho_bar;       // current rho-bar (Section 5.2)
  double obj, prim_res, dual_res, eps_prim, eps_dual;
  double prs, drs, pnorm, dnorm;   // scaled residuals / normalisers of the last check
  double solve_ms;      // device wall time of this QP's solve
  double polish_ms;     // device wall time of its polishing step
  double factor_rho;    // rho-bar the stored dense factor belongs to (0: none)
  double t_factor_ms, t_pcg_ms, t_update_ms, t_check_ms;   // device time per phase
  int status, iter, pcg_iter, rho_updates, polish_status;
  int init_mode;        // 0 continue, 1 zeros, 2 warm start from xws/yws
  int bad;              // internal failure flag (non-finite PCG scalar etc.)
  int pad;
};

// Settings as the kernels see them.
struct DevSettings {
  double sigma, alpha, eps_abs, eps_rel, eps_pinf, eps_dinf, delta, time_limit;
  double pcg_tol_frac;
  double wall_tick_s;   // seconds per wall_clock64() tick
  int max_iter, check_every, scaling_iters, adaptive_rho, polish, refine, pcg_max_iter;
  int pad;
};

// Device pointers of a batch.  T is the working precision of the ADMM/PCG
// loop; every *64 array is double.
template <class T>
struct Batch {
  const QPDesc *desc;
  QPState *st;
  int nq;
  const int *order;   // solve order (largest first)
  int *counter;       // work-queue head
  // patterns (shared by every value array of the same matrix)
  const int *a_rp, *a_ci, *at_rp, *at_ci, *p_rp, *p_ci;
  // unscaled data (double)
  const double *a_raw, *at_raw, *p_raw, *q_raw, *l_raw, *u_raw;
  // scaled data
  T *a_v, *at_v, *p_v, *q, *l, *u, *pdiag;
  double *a64, *at64, *p64, *q64, *l64, *u64;
  double *D, *E, *Dinv, *Einv;
  const unsigned char *is_eq;
  // iterates and work vectors
  T *rho, *rhoinv, *minv;
  double *x, *z, *y, *xt;   // ADMM iterates (double in both modes)
  T *zt, *r, *d, *p, *w, *t, *s;   // PCG work vectors in the working precision
  double *dx, *dy;
  double *zt64, *s64;
  const double *xws, *yws;
  double *xo, *yo, *zo;
  // dense path: factors, per-workgroup rank-k scratch, multi-entry rows
  T *dmat;
  T *dws;
  long long dws_stride;
  // low-rank path (FP64): per-QP blocks [Delta^-1 | u | S^-1 | w (compact) |
  // w (by row)] and per-workgroup scratch (G, then the inverse's panels)
  double *lmat;
  double *lws;
  long long lws_stride;
  const int *mrows;
  // band path: position -> variable and variable -> position, n-vector layout
  const int *bperm, *biperm;
  DevSettings set;
};

}  // namespace osqpmi
