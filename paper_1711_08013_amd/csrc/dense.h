// Workgroup-level dense linear algebra on row-major matrices in global
// memory (lower triangle used): blocked right-looking Cholesky with LDS
// tiles, forward/backward triangular solves, and the symmetric rank-k
// update M += s B'B.  Used by the FP64 polishing step (Section 4) and the
// dense small-QP path.  One workgroup owns one matrix; every routine ends
// with a barrier so results are visible to the whole workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include "team.h"

namespace osqpmi {

constexpr int kNB = 32;   // Cholesky panel width
constexpr int kTS = 64;   // trailing-update tile (kTS x kTS outputs)

// LDS of the dense routines.  The factorisation tiles and the diagonal
// block of a triangular solve are never live at the same time and share
// storage, which keeps the FP64 instance near 43 KB.
template <class T>
struct DenseLDS {
  union {
    struct {
      T pa[kTS][kNB + 1];
      T pb[kTS][kNB + 1];
      T diag[kNB][kNB + 1];
    };
    struct {
      T blk[64][65];   // a diagonal block of L
      T xs[64][65];    // its inverse, row by row
    };
  };
  T ys[64];
  int flag;
};

// Doubles of LDS a workgroup may use to stage a gathered vector; the stage
// overlays the factorisation tiles of DenseLDS<double> (never live at the
// same time) and stays clear of its ys and flag, which the triangular solve
// uses while a stage is live.
constexpr int kStage = 8192;
static_assert(kStage * sizeof(double) <= 2 * 64 * 65 * sizeof(double), "stage overlaps ys");

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output row of register v of lane group lk (= lane / 16) of a 16x16x4
// MFMA: the FP32 instruction returns D[4 lk + v][lane % 16], the FP64 one
// D[lk + 4 v][lane % 16] (both take A[lane % 16][lane / 16] and
// B[lane / 16][lane % 16]).
template <class T>
__device__ __forceinline__ int mfma_row(int lk, int v) {
  return sizeof(T) == 4 ? 4 * lk + v : lk + 4 * v;
}

// C[i0.., j0..] += scale * Pa Pb' for one kTS x kTS tile, depth kd <= kNB
// (Pa holds the i rows, Pb the j rows, both in LDS, zero-padded to kNB).
// Matrix cores: each of the first four waves owns four 16 x 16 output
// sub-tiles and runs 16x16x4 MFMAs over the depth (layout as mfma_row).
template <class T>
__device__ __forceinline__ void tile_gemm_nt_mfma(const WGTeam &tm, DenseLDS<T> &s, T *C, int ld,
                                                  int i0, int j0, int ni, int nj, int kd,
                                                  T scale, bool lower_only) {
  typedef T vec4 __attribute__((ext_vector_type(4)));
  const int wv = tm.tid >> 6, lane = tm.tid & 63;
  if (wv >= 4) return;
  const int li = lane & 15, lk = lane >> 4;
  const int kpad = (kd + 3) & ~3;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int sub = wv * 4 + q;            // 16 sub-tiles of the 64 x 64 tile
    const int si = (sub >> 2) * 16, sj = (sub & 3) * 16;
    vec4 acc = {T(0), T(0), T(0), T(0)};
    for (int k0 = 0; k0 < kpad; k0 += 4)
      acc = mfma16x16x4(s.pa[si + li][k0 + lk], s.pb[sj + li][k0 + lk], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = si + mfma_row<T>(lk, v), j = sj + li;
      if (i >= ni || j >= nj) continue;
      if (lower_only && i0 + i < j0 + j) continue;
      C[(size_t)(i0 + i) * ld + (j0 + j)] += scale * acc[v];
    }
  }
}

// Same tile update on the vector ALUs.
template <class T>
__device__ __forceinline__ void tile_gemm_nt_valu(const WGTeam &tm, DenseLDS<T> &s, T *C,
                                                  int ld, int i0, int j0, int ni, int nj, int kd,
                                                  T scale, bool lower_only) {
  for (int blk = tm.tid; blk < (kTS / 4) * (kTS / 4); blk += tm.nt) {
    const int bi = (blk / (kTS / 4)) * 4, bj = (blk % (kTS / 4)) * 4;
    T acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
    for (int t = 0; t < kd; ++t) {
      T va[4], vb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) { va[a] = s.pa[bi + a][t]; vb[a] = s.pb[bj + a][t]; }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += va[a] * vb[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = bi + a;
      if (i >= ni) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = bj + b;
        if (j >= nj) continue;
        if (lower_only && i0 + i < j0 + j) continue;
        C[(size_t)(i0 + i) * ld + (j0 + j)] += scale * acc[a][b];
      }
    }
  }
}

template <class T>
__device__ __forceinline__ void tile_gemm_nt(const WGTeam &tm, DenseLDS<T> &s, T *C, int ld,
                                             int i0, int j0, int ni, int nj, int kd, T scale,
                                             bool lower_only) {
  if (tm.nt >= 4 * kWave)
    tile_gemm_nt_mfma<T>(tm, s, C, ld, i0, j0, ni, nj, kd, scale, lower_only);
  else
    tile_gemm_nt_valu<T>(tm, s, C, ld, i0, j0, ni, nj, kd, scale, lower_only);
}

// M (n x n, lower) += scale * B' B with B dense, nr x n, row-major (ldb).
template <class T>
__device__ __forceinline__ void dense_syrk_tn(const WGTeam &tm, DenseLDS<T> &s, T *M, int ld, const T *B,
                             int ldb, int nr, int n, T scale) {
  for (int i0 = 0; i0 < n; i0 += kTS) {
    const int ni = min(kTS, n - i0);
    for (int j0 = 0; j0 <= i0; j0 += kTS) {
      const int nj = min(kTS, n - j0);
      for (int r0 = 0; r0 < nr; r0 += kNB) {
        const int kd = min(kNB, nr - r0);
        for (int e = tm.tid; e < kTS * kNB; e += tm.nt) {
          const int row = e % kTS, t = e / kTS;
          s.pa[row][t] = (row < ni && t < kd) ? B[(size_t)(r0 + t) * ldb + i0 + row] : T(0);
          s.pb[row][t] = (row < nj && t < kd) ? B[(size_t)(r0 + t) * ldb + j0 + row] : T(0);
        }
        tm.sync();
        tile_gemm_nt(tm, s, M, ld, i0, j0, ni, nj, kd, scale, i0 == j0);
        tm.sync();
      }
    }
  }
}

// S (R x R, lower triangle written) = G G' for G dense R x K, row-major
// (ldg), FP64 on the vector ALUs.  64 x 64 output tiles from 64-wide k
// panels staged in LDS (the triangular-solve block area); 256 virtual
// threads own a 4 x 4 block of a tile each (rows ti + 16a, columns
// tj + 16c), so per k step a thread reads eight LDS values for sixteen FMAs.
// Workgroups of fewer than 256 threads take several passes over a tile.
__device__ __forceinline__ void dense_gram_lower_64(const WGTeam &tm, DenseLDS<double> &s,
                                                    const double *G, int ldg, int R, int K,
                                                    double *S, int ldS) {
  constexpr int KC = 64;
  const int passes = tm.nt >= 256 ? 1 : (256 + tm.nt - 1) / tm.nt;
  for (int i0 = 0; i0 < R; i0 += kTS) {
    const int ni = min(kTS, R - i0);
    for (int j0 = 0; j0 <= i0; j0 += kTS) {
      const int nj = min(kTS, R - j0);
      for (int ps = 0; ps < passes; ++ps) {
        const int vt = tm.tid + ps * tm.nt;
        const bool act = vt < 256;
        const int ti = (vt >> 4) & 15, tj = vt & 15;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
        for (int k0 = 0; k0 < K; k0 += KC) {
          const int kd = min(KC, K - k0);
          tm.sync();
          for (int e = tm.tid; e < kTS * KC; e += tm.nt) {
            const int r = e / KC, t = e % KC;
            s.blk[r][t] = (r < ni && t < kd) ? G[(size_t)(i0 + r) * ldg + k0 + t] : 0.0;
            s.xs[r][t] = (r < nj && t < kd) ? G[(size_t)(j0 + r) * ldg + k0 + t] : 0.0;
          }
          tm.sync();
          if (act) {
#pragma unroll 4
            for (int t = 0; t < KC; ++t) {
              double av[4], bv[4];
#pragma unroll
              for (int a = 0; a < 4; ++a) av[a] = s.blk[ti + 16 * a][t];
#pragma unroll
              for (int c = 0; c < 4; ++c) bv[c] = s.xs[tj + 16 * c][t];
#pragma unroll
              for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] += av[a] * bv[c];
            }
          }
        }
        if (act) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int i = ti + 16 * a, j = tj + 16 * c;
              if (i < ni && j < nj && i0 + i >= j0 + j) S[(size_t)(i0 + i) * ldS + j0 + j] = acc[a][c];
            }
        }
      }
    }
  }
  tm.sync();
}

// The same product for R <= min(240, nt / 2) (nt >= 256 threads): each
// 16-deep k panel holds all R rows in LDS, so G is read once per pass
// instead of once per output tile; the lower 16 x 16 sub-tiles are dealt to
// the waves, at most four per wave and pass (their accumulators stay in
// registers), FP64 16x16x4 MFMAs.  The next panel is loaded into registers
// (16-byte loads: ldg a multiple of 2, rows 16-byte aligned, readable up to
// column K rounded up to 2) while the current one is used.
constexpr int kGramPanelMaxR = 240;
__device__ __forceinline__ void dense_gram_lower_panel(const WGTeam &tm, DenseLDS<double> &s,
                                                       const double *G, int ldg, int R, int K,
                                                       double *S, int ldS) {
  constexpr int KC = 16, LDP = KC + 1, QW = 4, NP = 4;   // 8 R <= NP nt (see the dispatch)
  static_assert(kGramPanelMaxR * LDP <= 2 * 64 * 65, "gram panel exceeds the block area");
  double *P = &s.blk[0][0];
  const int wv = tm.tid >> 6, nw = tm.nt >> 6, lane = tm.tid & (kWave - 1);
  const int li = lane & 15, lk = lane >> 4;
  const int nbk = (R + 15) / 16, T = nbk * (nbk + 1) / 2, npair = R * (KC / 2);
  constexpr int PS = KC / 2;   // 16-byte pairs per panel row
  for (int p0 = 0; p0 < T; p0 += nw * QW) {
    int bi[QW], bj[QW];
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int idx = p0 + wv + nw * q;   // uniform in the wave
      int r = 0;
      while ((r + 1) * (r + 2) / 2 <= idx) ++r;
      bi[q] = idx < T ? r : -1;
      bj[q] = idx - r * (r + 1) / 2;
    }
    f64x4 acc[QW];
#pragma unroll
    for (int q = 0; q < QW; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
    double2 nxt[NP];
    auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int e = tm.tid + tm.nt * u, r = e / PS, t = 2 * (e % PS);
        double2 x = {0.0, 0.0};
        if (e < npair && k0 + t < K) {
          x = *reinterpret_cast<const double2 *>(G + (size_t)r * ldg + k0 + t);
          if (k0 + t + 1 >= K) x.y = 0.0;
        }
        nxt[u] = x;
      }
    };
    load(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
      tm.sync();
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int e = tm.tid + tm.nt * u, r = e / PS, t = 2 * (e % PS);
        if (e < npair) {
          P[r * LDP + t] = nxt[u].x;
          P[r * LDP + t + 1] = nxt[u].y;
        }
      }
      tm.sync();
      if (k0 + KC < K) load(k0 + KC);
#pragma unroll
      for (int q = 0; q < QW; ++q) {
        if (bi[q] < 0) continue;
        // rows past R read stale LDS: they only reach output rows and
        // columns past R, which are not written
        const double *pa = P + min(16 * bi[q] + li, R - 1) * LDP + lk;
        const double *pb = P + min(16 * bj[q] + li, R - 1) * LDP + lk;
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) acc[q] = mfma16x16x4(pa[kk], pb[kk], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      if (bi[q] < 0) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * bi[q] + mfma_row<double>(lk, v), j = 16 * bj[q] + li;
        if (i < R && j < R && i >= j) S[(size_t)i * ldS + j] = acc[q][v];
      }
    }
  }
  tm.sync();
}

__device__ __forceinline__ void dense_gram_lower(const WGTeam &tm, DenseLDS<double> &s,
                                                 const double *G, int ldg, int R, int K,
                                                 double *S, int ldS) {
  if (tm.nt >= 4 * kWave && R <= kGramPanelMaxR && 2 * R <= tm.nt)
    dense_gram_lower_panel(tm, s, G, ldg, R, K, S, ldS);
  else dense_gram_lower_64(tm, s, G, ldg, R, K, S, ldS);
}

// In-place Cholesky M = L L' of the lower triangle.  Returns false (to every
// thread) when a pivot is not positive or not finite.
template <class T>
__device__ __forceinline__ bool dense_cholesky(const WGTeam &tm, DenseLDS<T> &s, T *M, int ld, int n) {
  if (tm.tid == 0) s.flag = 0;
  tm.sync();
  for (int kb = 0; kb < n; kb += kNB) {
    const int nb = min(kNB, n - kb);
    // (a) diagonal block into LDS and unblocked factorisation
    for (int e = tm.tid; e < kNB * kNB; e += tm.nt) {
      const int r = e / kNB, c = e % kNB;
      s.diag[r][c] = (r < nb && c <= r) ? M[(size_t)(kb + r) * ld + kb + c] : T(0);
    }
    tm.sync();
    // wave 0 factors the block in registers: lane r holds row r
    if (tm.tid < kWave) {
      const int r = tm.tid;
      T row[kNB];
#pragma unroll
      for (int c = 0; c < kNB; ++c) row[c] = (r < nb && c <= r) ? s.diag[r][c] : T(0);
      bool bad = false;
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        if (c < nb) {
          const T piv = __shfl(row[c], c, kWave);
          bad |= !(piv > T(0)) || !isfinite(double(piv));
          const T d = piv > T(0) ? T(sqrt(double(piv))) : T(1);
          if (r == c) row[c] = d;
          else if (r > c) row[c] = row[c] / d;
#pragma unroll
          for (int q = c + 1; q < kNB; ++q) {
            const T lqc = __shfl(row[c], q, kWave);
            if (q < nb && r >= q) row[q] -= row[c] * lqc;
          }
        }
      }
      if (r < nb) {
#pragma unroll
        for (int c = 0; c < kNB; ++c)
          if (c <= r) s.diag[r][c] = row[c];
      }
      if (r == 0 && bad) s.flag = 1;
    }
    tm.sync();
    for (int e = tm.tid; e < nb * nb; e += tm.nt) {
      const int r = e / nb, c = e % nb;
      if (c <= r) M[(size_t)(kb + r) * ld + kb + c] = s.diag[r][c];
    }
    // (b) panel: each row below solves x L_kk' = M_row in place (its own
    // nb entries stay in cache; no register array)
    for (int i = kb + nb + tm.tid; i < n; i += tm.nt) {
      T *row = M + (size_t)i * ld + kb;
      for (int c = 0; c < nb; ++c) {
        T v = row[c];
        for (int q = 0; q < c; ++q) v -= row[q] * s.diag[c][q];
        row[c] = v / s.diag[c][c];
      }
    }
    tm.sync();
    // (c) trailing update of the lower triangle: M22 -= L21 L21'
    const int t0 = kb + nb;
    for (int i0 = t0; i0 < n; i0 += kTS) {
      const int ni = min(kTS, n - i0);
      for (int j0 = t0; j0 <= i0; j0 += kTS) {
        const int nj = min(kTS, n - j0);
        for (int e = tm.tid; e < kTS * kNB; e += tm.nt) {
          const int row = e / kNB, t = e % kNB;
          s.pa[row][t] = (row < ni && t < nb) ? M[(size_t)(i0 + row) * ld + kb + t] : T(0);
          s.pb[row][t] = (row < nj && t < nb) ? M[(size_t)(j0 + row) * ld + kb + t] : T(0);
        }
        tm.sync();
        tile_gemm_nt(tm, s, M, ld, i0, j0, ni, nj, nb, T(-1), i0 == j0);
        tm.sync();
      }
    }
  }
  tm.sync();
  const bool ok = s.flag == 0;
  tm.sync();
  return ok;
}

constexpr int kSB = 64;   // triangular-solve block

// Inverses of the 64 x 64 diagonal blocks of L (row-major, lower), stored as
// nblk consecutive 64 x 64 row-major blocks in Linv (zero above the
// diagonal).  Wave 0 forms each inverse row by row in LDS: row r of X = L_kk^-1
// is (e_r - sum_{q<r} L_rq X_q) / L_rr, one column per lane.
template <class T>
__device__ __forceinline__ void dense_invert_diag(const WGTeam &tm, DenseLDS<T> &s, const T *L,
                                                  int ld, int n, T *Linv) {
  const int nblk = (n + kSB - 1) / kSB;
  const int lane = tm.tid & (kWave - 1);
  for (int bk = 0; bk < nblk; ++bk) {
    const int kb = bk * kSB, nb = min(kSB, n - kb);
    for (int e = tm.tid; e < kSB * kSB; e += tm.nt) {
      const int r = e / kSB, c = e % kSB;
      // padded rows/columns beyond nb: identity, so the padded inverse is too
      s.blk[r][c] = (r < nb && c <= r) ? L[(size_t)(kb + r) * ld + kb + c]
                                        : (r == c ? T(1) : T(0));
    }
    tm.sync();
    if (tm.tid < kWave) {
      const int c = lane;
      for (int r = 0; r < kSB; ++r) {
        T v = (r == c) ? T(1) : T(0);
        for (int q = c; q < r; ++q) v -= s.blk[r][q] * s.xs[q][c];
        s.xs[r][c] = (c <= r) ? v / s.blk[r][r] : T(0);
      }
    }
    tm.sync();
    T *dst = Linv + (size_t)bk * kSB * kSB;
    for (int e = tm.tid; e < kSB * kSB; e += tm.nt) dst[e] = s.xs[e / kSB][e % kSB];
    tm.sync();
  }
}

// C (ni x nj, row-major, ldc) += scale * A B' with A (ni x K) and B (nj x K)
// row-major (lda, ldb), ni, nj <= kTS: depth panels of kNB staged in LDS,
// the matrix-core tile product.
__device__ __forceinline__ void tile_nt_acc(const WGTeam &tm, DenseLDS<double> &s, double *C,
                                            int ldc, const double *A, int lda, const double *B,
                                            int ldb, int ni, int nj, int K, double scale) {
  for (int k0 = 0; k0 < K; k0 += kNB) {
    const int kd = min(kNB, K - k0);
    for (int e = tm.tid; e < kTS * kNB; e += tm.nt) {
      const int r = e / kNB, t = e % kNB;
      s.pa[r][t] = (r < ni && t < kd) ? A[(size_t)r * lda + k0 + t] : 0.0;
      s.pb[r][t] = (r < nj && t < kd) ? B[(size_t)r * ldb + k0 + t] : 0.0;
    }
    tm.sync();
    tile_gemm_nt<double>(tm, s, C, ldc, 0, 0, ni, nj, kd, scale, false);
    tm.sync();
  }
}

// Doubles of scratch dense_spd_inverse needs besides U (R x ld).
__host__ __device__ inline int64_t spd_inverse_extra(int R) {
  return (int64_t)((R + 63) / 64 + 1) * 4096;
}

// Inverse of an SPD matrix from its Cholesky factor: S (R x R, row-major, ld
// a multiple of 8, the factor L in its lower triangle) is overwritten by the
// full symmetric S^-1 (zero in the padding columns R..ld-1).  Scratch: U
// (R x ld) and `work` (spd_inverse_extra(R) doubles).  With 64 x 64 blocks,
// U = (L^-1)' is built block row by block row: U_jj = (L_jj^-1)' from the
// inverted diagonal blocks, and for i > j
//     U_ji = -(sum_{k=j..i-1} U_jk L_ik') (L_ii^-1)'
// (the transpose of the block forward substitution for L X = I).  Then
// S^-1 = L^-T L^-1 = U U' (lower triangle by the Gram routine, mirrored).
__device__ __forceinline__ void dense_spd_inverse(const WGTeam &tm, DenseLDS<double> &s, double *S,
                                                  int ld, int R, double *U, double *work) {
  const int nb = (R + 63) / 64;
  double *Linv = work, *W = work + (size_t)nb * 4096;
  dense_invert_diag<double>(tm, s, S, ld, R, Linv);
  for (size_t e = tm.tid; e < (size_t)R * ld; e += tm.nt) U[e] = 0.0;
  tm.sync();
  for (int j = 0; j < nb; ++j) {
    const int j0 = 64 * j, nj = min(64, R - j0);
    const double *Lj = Linv + (size_t)j * 4096;
    for (int e = tm.tid; e < nj * nj; e += tm.nt) {
      const int a = e / nj, b = e % nj;
      U[(size_t)(j0 + a) * ld + j0 + b] = Lj[b * 64 + a];
    }
    tm.sync();
    for (int i = j + 1; i < nb; ++i) {
      const int i0 = 64 * i, ni = min(64, R - i0);
      for (int e = tm.tid; e < 4096; e += tm.nt) W[e] = 0.0;
      tm.sync();
      for (int k = j; k < i; ++k)   // blocks k < i are full (64 wide)
        tile_nt_acc(tm, s, W, 64, U + (size_t)j0 * ld + 64 * k, ld, S + (size_t)i0 * ld + 64 * k,
                    ld, nj, ni, 64, 1.0);
      tile_nt_acc(tm, s, U + (size_t)j0 * ld + i0, ld, W, 64, Linv + (size_t)i * 4096, 64, nj, ni,
                  ni, -1.0);
    }
  }
  dense_gram_lower(tm, s, U, ld, R, R, S, ld);
  // upper triangle from the lower one (only upper entries are written)
  for (size_t e = tm.tid; e < (size_t)R * ld; e += tm.nt) {
    const int i = (int)(e / ld), j = (int)(e % ld);
    if (j > i) S[e] = j < R ? S[(size_t)j * ld + i] : 0.0;
  }
  tm.sync();
}

// f(r, sum_c M[r][c] y[c]) for the R rows of a dense matrix (row-major, ld
// a multiple of 8, rows 16-byte aligned, readable up to column ld-1; y
// readable up to index R rounded up to 8).  A wave takes four rows at a
// time, each lane two columns per 16-byte load and row, so all of a lane's
// loads for the four rows are in flight together; fixed summation order.
template <class F>
__device__ __forceinline__ void dense_rows_matvec(const WGTeam &tm, const double *M, int ld, int R,
                                                  const double *y, F &&f) {
  constexpr int RU = 4;
  const int lane = tm.tid & (kWave - 1), wv = tm.tid >> 6, nw = tm.nt >> 6;
  for (int r0 = RU * wv; r0 < R; r0 += RU * nw) {
    double acc[RU];
#pragma unroll
    for (int q = 0; q < RU; ++q) acc[q] = 0.0;
    // 256 columns per step: two 16-byte loads per lane and row, all issued
    // before any is used
    for (int c0 = 0; c0 < R; c0 += 4 * kWave) {
      double2 mv[RU][2];
      double yv[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = min(c0 + 2 * lane + 2 * kWave * h, (R - 1) & ~1);
#pragma unroll
        for (int q = 0; q < RU; ++q)
          mv[q][h] = *reinterpret_cast<const double2 *>(M + (size_t)min(r0 + q, R - 1) * ld + c);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = c0 + 2 * lane + 2 * kWave * h;
        yv[2 * h] = c < R ? y[c] : 0.0;
        yv[2 * h + 1] = c + 1 < R ? y[c + 1] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < RU; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[q] += mv[q][h].x * yv[2 * h] + mv[q][h].y * yv[2 * h + 1];
    }
#pragma unroll
    for (int q = 0; q < RU; ++q) {
      const double t = group_sum(acc[q], kWave);
      if (lane == 0 && r0 + q < R) f(r0 + q, t);
    }
  }
}

// Four consecutive T from a 16-byte-aligned address.
template <class T>
__device__ __forceinline__ void load4(const T *p, T &a, T &b, T &c, T &d) {
  if constexpr (sizeof(T) == 4) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
  } else {
    const double2 v0 = *reinterpret_cast<const double2 *>(p);
    const double2 v1 = *reinterpret_cast<const double2 *>(p + 2);
    a = v0.x; b = v0.y; c = v1.x; d = v1.y;
  }
}

// Solve L L' x = b in place (b -> x); L lower, row-major (ld a multiple of 8),
// Linv the inverted diagonal blocks.  Per 64-row block: the block unknowns
// are a 64 x 64 matrix-vector product with the block inverse (parallel), then
// the rest of the workgroup's rows / columns are updated.  The forward sweep
// reads L by 64-wide row chunks (16 lanes per row, 16-byte loads, several
// rows in flight), the backward sweep by column quads (64 rows in flight per
// lane), so each sweep reads the lower triangle once.
template <class T>
__device__ __forceinline__ void dense_solve_llt(const WGTeam &tm, DenseLDS<T> &s, const T *L,
                                                int ld, int n, const T *Linv, T *x) {
  const int nblk = (n + kSB - 1) / kSB;
  // ---- forward: L y = b
  for (int bk = 0; bk < nblk; ++bk) {
    const int kb = bk * kSB, nb = min(kSB, n - kb);
    const T *Bi = Linv + (size_t)bk * kSB * kSB;
    // y_blk = Linv_kk b_blk: 4 lanes per row, 16 columns each
    for (int t = tm.tid; t < kSB * 4; t += tm.nt) {
      const int r = t >> 2, part = t & 3;
      T acc = T(0);
      if (r < nb) {
#pragma unroll
        for (int c4 = 0; c4 < 16; c4 += 4) {
          const int c = part * 16 + c4;
          T a0, a1, a2, a3;
          load4(Bi + r * kSB + c, a0, a1, a2, a3);
          acc += (c + 0 < nb ? a0 * x[kb + c + 0] : T(0)) + (c + 1 < nb ? a1 * x[kb + c + 1] : T(0)) +
                 (c + 2 < nb ? a2 * x[kb + c + 2] : T(0)) + (c + 3 < nb ? a3 * x[kb + c + 3] : T(0));
        }
      }
      acc = group_sum(acc, 4);
      if (part == 0) s.ys[r] = acc;
    }
    tm.sync();
    for (int r = tm.tid; r < nb; r += tm.nt) x[kb + r] = s.ys[r];
    // rows below: b_i -= L[i, kb:kb+64] y_blk (only when a full block is above)
    if (kb + nb < n) {
      const int sub = tm.tid & 15, grp = tm.tid >> 4, ngrp = tm.nt >> 4;
      const T y0 = s.ys[4 * sub], y1 = s.ys[4 * sub + 1], y2 = s.ys[4 * sub + 2],
              y3 = s.ys[4 * sub + 3];
      constexpr int U = 4;
      for (int i0 = kb + nb + grp; i0 < n; i0 += ngrp * U) {
        T part[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * ngrp;
          part[u] = T(0);
          if (i < n) {
            T a0, a1, a2, a3;
            load4(L + (size_t)i * ld + kb + 4 * sub, a0, a1, a2, a3);
            part[u] = a0 * y0 + a1 * y1 + a2 * y2 + a3 * y3;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const T v = group_sum(part[u], 16);
          const int i = i0 + u * ngrp;
          if (sub == 0 && i < n) x[i] -= v;
        }
      }
    }
    tm.sync();
  }
  // ---- backward: L' x = y
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int kb = bk * kSB, nb = min(kSB, n - kb);
    const T *Bi = Linv + (size_t)bk * kSB * kSB;
    // x_blk = Linv_kk' y_blk: x_c = sum_{r >= c} Linv[r][c] y_r
    for (int t = tm.tid; t < kSB * 4; t += tm.nt) {
      const int c = t >> 2, part = t & 3;
      T acc = T(0);
      if (c < nb) {
        for (int r = part * 16; r < part * 16 + 16; ++r)
          if (r >= c && r < nb) acc += Bi[r * kSB + c] * x[kb + r];
      }
      acc = group_sum(acc, 4);
      if (part == 0) s.ys[c] = acc;
    }
    tm.sync();
    for (int r = tm.tid; r < nb; r += tm.nt) x[kb + r] = s.ys[r];
    // columns to the left: x_j -= sum_r L[kb+r, j] x_{kb+r}, j < kb, four
    // columns per thread, the 64 rows' loads in flight together
    for (int j = 4 * tm.tid; j < kb; j += 4 * tm.nt) {
      T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll 16
      for (int r = 0; r < kSB; ++r) {
        if (r < nb) {
          T l0, l1, l2, l3;
          load4(L + (size_t)(kb + r) * ld + j, l0, l1, l2, l3);
          const T yr = s.ys[r];
          a0 += l0 * yr; a1 += l1 * yr; a2 += l2 * yr; a3 += l3 * yr;
        }
      }
      x[j] -= a0; x[j + 1] -= a1; x[j + 2] -= a2; x[j + 3] -= a3;
    }
    tm.sync();
  }
}

}  // namespace osqpmi
