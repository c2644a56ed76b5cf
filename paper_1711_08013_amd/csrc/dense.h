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

template <class T>
struct DenseLDS {
  T pa[kTS][kNB + 1];
  T pb[kTS][kNB + 1];
  T diag[kNB][kNB + 1];
  int flag;
};

// C[I.., J..] -= Pa Pb' for one kTS x kTS tile, depth kd <= kNB, where Pa rows
// come from the i-range and Pb rows from the j-range (already in LDS).
// 256 threads: each owns a 4 x 4 block of the tile.
template <class T>
__device__ __forceinline__ void tile_gemm_nt(const WGTeam &tm, DenseLDS<T> &s, T *C, int ld,
                                             int i0, int j0, int ni, int nj, int kd,
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

// M (n x n, lower) += scale * B' B with B dense, nr x n, row-major (ldb).
template <class T>
__device__ void dense_syrk_tn(const WGTeam &tm, DenseLDS<T> &s, T *M, int ld, const T *B,
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
__device__ bool dense_cholesky(const WGTeam &tm, DenseLDS<T> &s, T *M, int ld, int n) {
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
    // (b) panel: rows below solve x L_kk' = M_row
    for (int i = kb + nb + tm.tid; i < n; i += tm.nt) {
      T *row = M + (size_t)i * ld + kb;
      T x[kNB];
#pragma unroll
      for (int c = 0; c < kNB; ++c) x[c] = c < nb ? row[c] : T(0);
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        if (c < nb) {
          T v = x[c];
#pragma unroll
          for (int q = 0; q < kNB; ++q)
            if (q < c) v -= x[q] * s.diag[c][q];
          x[c] = v / s.diag[c][c];
        }
      }
#pragma unroll
      for (int c = 0; c < kNB; ++c)
        if (c < nb) row[c] = x[c];
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

// Solve L y = b in place (b -> y).  L lower, row-major.
template <class T>
__device__ void dense_forward(const WGTeam &tm, DenseLDS<T> &s, const T *L, int ld, int n,
                              T *b) {
  for (int kb = 0; kb < n; kb += kNB) {
    const int nb = min(kNB, n - kb);
    // diagonal block by one thread (kNB x kNB)
    if (tm.tid == 0) {
      for (int c = 0; c < nb; ++c) {
        T v = b[kb + c];
        for (int q = 0; q < c; ++q) v -= L[(size_t)(kb + c) * ld + kb + q] * b[kb + q];
        b[kb + c] = v / L[(size_t)(kb + c) * ld + kb + c];
      }
    }
    tm.sync();
    // rows below: b_i -= L[i, kb:kb+nb] y_blk
    for (int i = kb + nb + tm.tid; i < n; i += tm.nt) {
      const T *row = L + (size_t)i * ld + kb;
      T acc = T(0);
      for (int c = 0; c < nb; ++c) acc += row[c] * b[kb + c];
      b[i] -= acc;
    }
    tm.sync();
  }
}

// Solve L' x = y in place (y -> x).
template <class T>
__device__ void dense_backward(const WGTeam &tm, DenseLDS<T> &s, const T *L, int ld, int n,
                               T *y) {
  const int nblk = (n + kNB - 1) / kNB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int kb = bk * kNB, nb = min(kNB, n - kb);
    // u_c = sum_{i >= kb+nb} L[i, kb+c] x_i, accumulated per thread then
    // combined through LDS (pa reused as [thread][c] partials in chunks)
    T part[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) part[c] = T(0);
    for (int i = kb + nb + tm.tid; i < n; i += tm.nt) {
      const T *row = L + (size_t)i * ld + kb;
      const T xi = y[i];
#pragma unroll
      for (int c = 0; c < kNB; ++c)
        if (c < nb) part[c] += row[c] * xi;
    }
    // reduce over the workgroup: waves shuffle, then LDS across waves
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
      T v = part[c];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
      part[c] = v;
    }
    const int wv = tm.tid >> 6, lane = tm.tid & 63;
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kNB; ++c) s.pa[wv][c] = part[c];
    }
    tm.sync();
    if (tm.tid == 0) {
      const int nw = tm.nt >> 6;
      for (int c = nb - 1; c >= 0; --c) {
        T u = T(0);
        for (int w = 0; w < nw; ++w) u += s.pa[w][c];
        // within the block: subtract L[kb+r, kb+c] x_{kb+r} for r > c
        for (int r = c + 1; r < nb; ++r) u += L[(size_t)(kb + r) * ld + kb + c] * y[kb + r];
        y[kb + c] = (y[kb + c] - u) / L[(size_t)(kb + c) * ld + kb + c];
      }
    }
    tm.sync();
  }
}

}  // namespace osqpmi
