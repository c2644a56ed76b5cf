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
    T blk[64][65];   // diagonal block of a triangular solve
  };
  T ys[64];
  int flag;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C[i0.., j0..] += scale * Pa Pb' for one kTS x kTS tile, depth kd <= kNB
// (Pa holds the i rows, Pb the j rows, both in LDS, zero-padded to kNB).
// Matrix cores: each of the first four waves owns four 16 x 16 output
// sub-tiles and runs 16x16x4 MFMAs over the depth.  Operand layout of the
// 16x16x4 instruction: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[4 (l / 16) + v][l % 16], v = 0..3.
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
      const int i = si + 4 * lk + v, j = sj + li;
      if (i >= ni || j >= nj) continue;
      if (lower_only && i0 + i < j0 + j) continue;
      C[(size_t)(i0 + i) * ld + (j0 + j)] += scale * acc[v];
    }
  }
}

// Same tile update on the vector ALUs (used for double: the FP64 16x16x4
// instruction's result layout differs from the FP32 one assumed above).
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
  if constexpr (sizeof(T) == 4)
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
    for (int c = 0; c < nb; ++c) {
      if (tm.tid == 0) {
        const T piv = s.diag[c][c];
        if (!(piv > T(0)) || !isfinite(double(piv))) s.flag = 1;
        s.diag[c][c] = piv > T(0) ? T(sqrt(double(piv))) : T(1);
      }
      tm.sync();
      const T dc = s.diag[c][c];
      for (int r = c + 1 + tm.tid; r < nb; r += tm.nt) s.diag[r][c] /= dc;
      tm.sync();
      const int w = nb - c - 1;
      for (int e = tm.tid; e < w * w; e += tm.nt) {
        const int r = c + 1 + e / w, q = c + 1 + e % w;
        if (q <= r) s.diag[r][q] -= s.diag[r][c] * s.diag[q][c];
      }
      tm.sync();
    }
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

constexpr int kSB = 64;   // triangular-solve block (one wave solves a block)

// Solve L L' x = b in place (b -> x); L lower, row-major (ld).  Each 64-row
// block is solved by wave 0 in registers (shuffle broadcasts), the rest of
// the workgroup applies the block to the remaining rows; the forward sweep
// reads L by row chunks, the backward sweep by coalesced column chunks, so
// each sweep reads the lower triangle once.
template <class T>
__device__ __forceinline__ void dense_solve_llt(const WGTeam &tm, DenseLDS<T> &s, const T *L, int ld, int n,
                                T *x) {
  const int lane = tm.tid & (kWave - 1);
  const bool w0 = tm.tid < kWave;
  // forward: L y = b
  for (int kb = 0; kb < n; kb += kSB) {
    const int nb = min(kSB, n - kb);
    for (int e = tm.tid; e < nb * kSB; e += tm.nt) {
      const int r = e / kSB, c = e % kSB;
      s.blk[r][c] = (c <= r && c < nb) ? L[(size_t)(kb + r) * ld + kb + c] : T(0);
    }
    tm.sync();
    if (w0) {
      T br = lane < nb ? x[kb + lane] : T(0);
      for (int c = 0; c < nb; ++c) {
        const T lrc = lane < nb ? s.blk[lane][c] : T(0);
        const T yc = __shfl(lane == c ? br / lrc : T(0), c, kWave);
        if (lane == c) br = yc;
        else if (lane > c) br -= lrc * yc;
      }
      if (lane < nb) { x[kb + lane] = br; s.ys[lane] = br; }
    }
    tm.sync();
    for (int i = kb + nb + tm.tid; i < n; i += tm.nt) {
      const T *r = L + (size_t)i * ld + kb;
      T acc = T(0);
      for (int c = 0; c < nb; ++c) acc += r[c] * s.ys[c];
      x[i] -= acc;
    }
    tm.sync();
  }
  // backward: L' x = y
  const int nblk = (n + kSB - 1) / kSB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int kb = bk * kSB, nb = min(kSB, n - kb);
    for (int e = tm.tid; e < nb * kSB; e += tm.nt) {
      const int r = e / kSB, c = e % kSB;
      s.blk[r][c] = (c <= r && c < nb) ? L[(size_t)(kb + r) * ld + kb + c] : T(0);
    }
    tm.sync();
    if (w0) {
      T bs = lane < nb ? x[kb + lane] : T(0);
      for (int r = nb - 1; r >= 0; --r) {
        const T lrs = lane < nb ? s.blk[r][lane] : T(0);   // L[r][lane]
        const T xr = __shfl(lane == r ? bs / lrs : T(0), r, kWave);
        if (lane == r) bs = xr;
        else if (lane < r) bs -= lrs * xr;
      }
      if (lane < nb) { x[kb + lane] = bs; s.ys[lane] = bs; }
    }
    tm.sync();
    for (int j = tm.tid; j < kb; j += tm.nt) {
      T acc = T(0);
      for (int r = 0; r < nb; ++r) acc += L[(size_t)(kb + r) * ld + j] * s.ys[r];
      x[j] -= acc;
    }
    tm.sync();
  }
}

}  // namespace osqpmi
