// Teams of threads that cooperate on one QP.
//
//  * WGTeam   : one workgroup; barriers are s_barrier, reductions go through
//               LDS.  Used for batched QPs (one QP per workgroup at a time).
//  * GridTeam : every workgroup of a cooperative launch; barriers are a
//               counter/generation barrier in global memory, reductions are
//               two-level (per-workgroup partials, then every wave reads all
//               partials in a fixed order).  Used for single large QPs.
//
// Both give every thread the same reduction results in the same order, so
// all control decisions taken from them are uniform over the team, and the
// results do not depend on which workgroup ran which QP.
#pragma once

#include <hip/hip_runtime.h>

namespace osqpmi {

constexpr int kWave = 64;
constexpr int kRedSlots = 32;   // values per reduction call

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
// Sum over an aligned group of L lanes (L a power of two <= 64).
__device__ __forceinline__ float group_sum(float v, int L) {
  for (int o = L >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
  return v;
}
__device__ __forceinline__ double group_sum(double v, int L) {
  for (int o = L >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
  return v;
}
__device__ __forceinline__ double group_max(double v, int L) {
  for (int o = L >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, L));
  return v;
}

struct WGTeam {
  int tid, nt;
  double *red;   // LDS, (nt/64) * kRedSlots doubles

  __device__ __forceinline__ void sync() const { __syncthreads(); }

  // In-place reduction of NS sums followed by NM maxima (NS + NM <= kRedSlots);
  // every thread receives the team-wide results.
  template <int NS, int NM>
  __device__ __forceinline__ void reduce(double *v) const {
    static_assert(NS + NM <= kRedSlots, "too many values");
    const int lane = tid & (kWave - 1), wv = tid >> 6, nw = nt >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = NS; k < NS + NM; ++k) v[k] = wave_max(v[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NS + NM; ++k) red[wv * kRedSlots + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) {
      double a = red[k];
      for (int w = 1; w < nw; ++w) {
        const double b = red[w * kRedSlots + k];
        a = k < NS ? a + b : fmax(a, b);
      }
      v[k] = a;
    }
    __syncthreads();
  }
};

// Global barrier state for GridTeam (zeroed by the host before launch).
struct GridBarrier {
  unsigned int count;
  unsigned int gen;
  unsigned int timeout;   // set when a wait exceeded its spin limit
  unsigned int pad;
};

struct GridTeam {
  int tid, nt;
  int nblocks, bid;
  double *red;            // LDS, (blockDim/64) * kRedSlots doubles
  double *partials;       // global, nblocks * kRedSlots * 2 (double-buffered)
  GridBarrier *bar;
  mutable int phase;      // alternates the partials buffer between reductions

  __device__ __forceinline__ void sync() const {
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      unsigned int g = __hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      unsigned int arrived = atomicAdd(&bar->count, 1u);
      if (arrived == (unsigned int)nblocks - 1u) {
        __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        // bounded wait: every workgroup of a cooperative launch is resident,
        // so the generation advances; the limit only guards against a
        // launch that broke that contract.  After one timeout no barrier
        // waits any more (the result is flagged as a device error).
        unsigned int spins = 0;
        while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
          if (__hip_atomic_load(&bar->timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
          __builtin_amdgcn_s_sleep(2);
          if (++spins > (1u << 24)) {
            atomicOr(&bar->timeout, 1u);
            break;
          }
        }
      }
      __threadfence();
    }
    __syncthreads();
  }

  template <int NS, int NM>
  __device__ __forceinline__ void reduce(double *v) const {
    static_assert(NS + NM <= kRedSlots, "too many values");
    const int lt = threadIdx.x;
    const int lane = lt & (kWave - 1), wv = lt >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = NS; k < NS + NM; ++k) v[k] = wave_max(v[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NS + NM; ++k) red[wv * kRedSlots + k] = v[k];
    }
    __syncthreads();
    double *part = partials + (size_t)(phase & 1) * nblocks * kRedSlots;
    phase ^= 1;
    if (lt < NS + NM) {
      const int k = lt;
      double a = red[k];
      for (int w = 1; w < nw; ++w) {
        const double b = red[w * kRedSlots + k];
        a = k < NS ? a + b : fmax(a, b);
      }
      part[(size_t)bid * kRedSlots + k] = a;
    }
    sync();
    // every wave combines all workgroup partials in the same fixed order
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) {
      double a = k < NS ? 0.0 : -INFINITY;
      for (int b = lane; b < nblocks; b += kWave) {
        const double x = part[(size_t)b * kRedSlots + k];
        a = k < NS ? a + x : fmax(a, x);
      }
      v[k] = k < NS ? wave_sum(a) : wave_max(a);
    }
    // the other partials buffer is written by the next reduction; the one
    // read here is not touched again until two reductions later, and a
    // barrier separates those
  }
};

}  // namespace osqpmi
