// Kernel entry points of osqp_mi.
#pragma once

#include "polish.h"
#include "solver_device.h"

namespace osqpmi {

constexpr int kMaxBlock = 512;

__global__ void reset_counters_kernel(int *counter, int ncounters, GridBarrier *bar) {
  const int i = threadIdx.x;
  if (i < ncounters) counter[i] = 0;
  if (bar && i == 0) { bar->count = 0; bar->gen = 0; bar->timeout = 0; }
}

// Work-queue loop: each workgroup takes the next QP index of `list`
// (counter slot `slot`) until the list is exhausted.
template <class F>
__device__ __forceinline__ void wg_queue(int *counter, int nlist, int &slot_val, F &&body) {
  for (;;) {
    if (threadIdx.x == 0) slot_val = atomicAdd(counter, 1);
    __syncthreads();
    const int qi = __builtin_amdgcn_readfirstlane(slot_val);   // uniform: scalar loads
    __syncthreads();
    if (qi >= nlist) break;
    body(qi);
  }
}

template <class T>
__global__ void __launch_bounds__(kMaxBlock) scale_wg_kernel(Batch<T> b, const int *list,
                                                             int nlist, int slot) {
  __shared__ double red[(kMaxBlock / kWave) * kRedSlots];
  __shared__ double stage[kStage];
  WGTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
  __shared__ int slot_val;
  wg_queue(b.counter + slot, nlist, slot_val, [&](int qi) __attribute__((always_inline)) {
    QPView<T> v(b, list[qi]);
    scale_qp<T>(tm, v, b.set, stage);
  });
}

template <class T>
__global__ void __launch_bounds__(kMaxBlock) rescale_vectors_wg_kernel(Batch<T> b, int k) {
  __shared__ double red[(kMaxBlock / kWave) * kRedSlots];
  WGTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
  QPView<T> v(b, k);
  rescale_vectors<T>(tm, v);
}

// LDS of the exact preconditioners: the dense path works in T, the low-rank
// path in double; a QP uses one of them, so they share storage.
template <class T>
struct SolveLDS {
  union {
    DenseLDS<T> t;
    DenseLDS<double> d;
    double stage[kStage];   // gathered vectors of the sparse passes
  };
};

template <class T>
__global__ void __launch_bounds__(kMaxBlock) solve_wg_kernel(Batch<T> b, const int *list,
                                                             int nlist, int slot) {
  __shared__ double red[(kMaxBlock / kWave) * kRedSlots];
  __shared__ SolveLDS<T> dl;
  WGTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
  T *dB = b.dws ? b.dws + (size_t)blockIdx.x * (size_t)b.dws_stride : nullptr;
  double *G = b.lws ? b.lws + (size_t)blockIdx.x * (size_t)b.lws_stride : nullptr;
  __shared__ int slot_val;
  wg_queue(b.counter + slot, nlist, slot_val, [&](int qi) __attribute__((always_inline)) {
    QPView<T> v(b, list[qi]);
    solve_qp<T>(tm, v, b.set, &dl.t, dB, dB != nullptr, &dl.d, G, G != nullptr, dl.stage);
  });
}

// FP64 polishing (Section 4), one QP per workgroup; workgroup b uses the
// b-th workspace slot.  QPs that did not reach "solved" are skipped.
constexpr int kPolishBlock = 512;
template <class T>
__global__ void __launch_bounds__(kPolishBlock) polish_wg_kernel(Batch<T> b, const int *list,
                                                                 int nlist, int slot, double *ws,
                                                                 long long stride, int rmax) {
  __shared__ double red[(kPolishBlock / kWave) * kRedSlots];
  __shared__ DenseLDS<double> dl;
  WGTeam tm{(int)threadIdx.x, (int)blockDim.x, red};
  double *mine = ws + (size_t)blockIdx.x * (size_t)stride;
  __shared__ int slot_val;
  wg_queue(b.counter + slot, nlist, slot_val, [&](int qi) __attribute__((always_inline)) {
    const int k = list[qi];
    if (b.st[k].status != 1) return;
    QPView<T> v(b, k);
    polish_qp<T>(tm, dl, v, b.set, mine, rmax, b.desc[k].plr != 0);
  });
}

// Cooperative (grid-team) variants: every workgroup works on QP list[0..nlist)
// one after another.
template <class T>
__global__ void __launch_bounds__(kMaxBlock) scale_grid_kernel(Batch<T> b, const int *list,
                                                               int nlist, double *partials,
                                                               GridBarrier *bar) {
  __shared__ double red[(kMaxBlock / kWave) * kRedSlots];
  GridTeam tm{(int)(blockIdx.x * blockDim.x + threadIdx.x), (int)(gridDim.x * blockDim.x),
              (int)gridDim.x, (int)blockIdx.x, red, partials, bar, 0};
  for (int qi = 0; qi < nlist; ++qi) {
    QPView<T> v(b, list[qi]);
    scale_qp<T>(tm, v, b.set);
  }
}

template <class T>
__global__ void __launch_bounds__(kMaxBlock) solve_grid_kernel(Batch<T> b, const int *list,
                                                               int nlist, double *partials,
                                                               GridBarrier *bar) {
  __shared__ double red[(kMaxBlock / kWave) * kRedSlots];
  GridTeam tm{(int)(blockIdx.x * blockDim.x + threadIdx.x), (int)(gridDim.x * blockDim.x),
              (int)gridDim.x, (int)blockIdx.x, red, partials, bar, 0};
  for (int qi = 0; qi < nlist; ++qi) {
    QPView<T> v(b, list[qi]);
    solve_qp<T>(tm, v, b.set);
  }
}

}  // namespace osqpmi
