// CPU stand-in for <hip/hip_runtime.h>, used only by the test build that
// runs the library's kernels on the host (tests/simt/build.py).
//
// Device code compiles as ordinary C++: kernels become functions, LDS
// variables become function statics in a section of their own, and every
// thread of a workgroup runs as a fiber (own stack, switched by a small
// register-save routine).  A fiber yields at a workgroup barrier, at each
// cross-lane operation (shuffles, ballots, 16x16x4 matrix products) and in
// a spin-wait; the scheduler resumes it when the operation can complete:
//   * a barrier completes when every live thread of the workgroup waits on it
//     (one that only part of the workgroup reaches is reported);
//   * a cross-lane operation completes when every live lane of its aligned
//     segment (the shuffle width, else the wave) waits at the same call
//     site; lanes elsewhere are still on a longer path to it, which is the
//     order in which a wave runs a divergent branch.
// Threads run in alternating ascending and descending order between
// synchronisation points.  The workgroups of an ordinary launch run in
// groups of SIMT_SIDE_BY_SIDE (environment, default 4) side by side, taken
// alternately from the top and the bottom of the grid (so a work queue hands
// its items to the highest and the lowest per-workgroup workspace slots at
// once); those of a cooperative launch all run side by side.  Workgroups
// that run side by side each have their own copy of the LDS section.
// The emulated device has SIMT_CU_COUNT compute units (build-time, default
// 256, as on gfx950); occupancy and static LDS size come from the resource
// usage the gfx950 build reports for each kernel (registered by the build).
// Device memory is host memory from malloc, so a host address sanitizer
// sees every device access.
#pragma once

#include <execinfo.h>
#include <signal.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define SIMT_ASAN 1
#endif
#endif
#ifdef SIMT_ASAN
#include <sanitizer/common_interface_defs.h>
#endif

// ---- qualifiers ------------------------------------------------------------
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
// LDS variables live in a section of their own, so that a cooperative
// launch (several workgroups side by side) can give each workgroup its own
// copy: the section is swapped when the scheduler moves to another workgroup
#define __shared__ static __attribute__((section("simt_lds")))
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct alignas(16) int4 { int x, y, z, w; };
struct alignas(16) float4 { float x, y, z, w; };
struct alignas(8) float2 { float x, y; };
struct alignas(16) double2 { double x, y; };

using std::fmax;
using std::fmin;
using std::isfinite;
using std::isinf;
using std::isnan;
using std::sqrt;
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }

// Fiber switch (x86-64 System V): push the callee-saved registers, store the
// stack pointer to *from, load `to`, pop them and return into the target.
extern "C" void simt_switch(void **from, void *to);
asm(R"(
  .text
  .p2align 4
  .globl simt_switch
  .hidden simt_switch
  .type simt_switch,@function
simt_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size simt_switch, .-simt_switch
)");

extern "C" char __start_simt_lds[] __attribute__((weak));
extern "C" char __stop_simt_lds[] __attribute__((weak));

namespace simt {

constexpr int kWaveLanes = 64;

enum State { RUN = 0, BARRIER = 1, WAVE = 2, DONE = 3 };
enum Kind { SHFL_XOR = 1, SHFL = 2, BALLOT = 3, MFMA64 = 4, MFMA32 = 5 };

struct Lane {
  int kind = 0, arg = 0, width = 0;
  const char *file = nullptr;   // call site of the pending cross-lane operation
  int line = 0;
  bool go = false;
  double v = 0.0, a = 0.0, b = 0.0, acc[4] = {0, 0, 0, 0};
  double r = 0.0, racc[4] = {0, 0, 0, 0};
  unsigned long long ur = 0;
  bool pred = false;
};

struct Fiber {
  void *sp = nullptr;      // saved stack pointer while switched out
  char *stack = nullptr;   // from the scheduler's pool
  State state = RUN;
  Lane lane;
};

struct Sched {
  std::vector<Fiber> f;
  std::vector<char *> stacks;   // kept across workgroups and launches
  void *main_sp = nullptr;
  const std::function<void()> *body = nullptr;
  int cur = -1, nt = 0, bid = 0, gdim = 1;
  unsigned long long clock = 0;
#ifdef SIMT_ASAN
  void *fake_main = nullptr;
  const void *main_bottom = nullptr;
  size_t main_size = 0;
#endif
};

inline Sched &S() {
  static Sched s;
  return s;
}

// threadIdx & co. read these (the scheduler keeps them current)
inline unsigned g_tid = 0, g_bid = 0, g_bdim = 1, g_gdim = 1;
struct DimRef {
  const unsigned &x;
  unsigned y, z;
};

// switch from the current fiber back to the scheduler
inline void yield_to_main() {
  Sched &s = S();
  Fiber &me = s.f[s.cur];
#ifdef SIMT_ASAN
  void *fake = nullptr;
  __sanitizer_start_switch_fiber(me.state == DONE ? nullptr : &fake, s.main_bottom, s.main_size);
#endif
  simt_switch(&me.sp, s.main_sp);
#ifdef SIMT_ASAN
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
}

inline void fiber_entry() {
  Sched &s = S();
#ifdef SIMT_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &s.main_bottom, &s.main_size);
#endif
  (*s.body)();
  s.f[s.cur].state = DONE;
  yield_to_main();
}

inline void wait(State st) {
  Sched &s = S();
  s.f[s.cur].state = st;
  yield_to_main();
}

// Complete the cross-lane operations of wave w that can complete: those
// whose aligned lane segment (the shuffle width; the whole wave for ballots
// and matrix products) has every live lane waiting at the same call site.
// Lanes of a segment that are elsewhere are still on their way there (a
// loop with more trips for them), as on hardware, where the wave runs the
// longer path first and meets again afterwards.  Returns whether any
// operation completed.
inline bool resolve_wave(int base, int end) {
  Sched &s = S();
  bool any = false;
  for (int t = base; t < end; ++t) s.f[t].lane.go = false;
  for (int t = base; t < end; ++t) {
    const Fiber &x = s.f[t];
    if (x.state != WAVE || x.lane.go) continue;
    const Lane &L = x.lane;
    const int width = (L.kind == SHFL_XOR || L.kind == SHFL) ? L.width : kWaveLanes;
    const int s0 = base + ((t - base) & ~(width - 1)), s1 = std::min(end, s0 + width);
    bool ok = true;
    for (int u = s0; u < s1 && ok; ++u) {
      const Fiber &y = s.f[u];
      if (y.state == DONE) continue;
      ok = y.state == WAVE && y.lane.kind == L.kind && y.lane.line == L.line &&
           y.lane.file == L.file && y.lane.width == L.width;
    }
    if (!ok) continue;
    for (int u = s0; u < s1; ++u)
      if (s.f[u].state == WAVE) s.f[u].lane.go = true;
    any = true;
  }
  if (!any) return false;
  unsigned long long bal = 0;
  for (int t = base; t < end; ++t)
    if (s.f[t].lane.go && s.f[t].lane.kind == BALLOT && s.f[t].lane.pred)
      bal |= 1ull << (t - base);
  for (int t = base; t < end; ++t) {
    Fiber &x = s.f[t];
    if (x.state != WAVE || !x.lane.go) continue;
    Lane &L = x.lane;
    const int l = t - base;
    switch (L.kind) {
      case SHFL_XOR: {
        const int src = (l & ~(L.width - 1)) | ((l ^ L.arg) & (L.width - 1));
        L.r = base + src < end ? s.f[base + src].lane.v : 0.0;
        break;
      }
      case SHFL: {
        const int src = (l & ~(L.width - 1)) + (L.arg & (L.width - 1));
        L.r = base + src < end ? s.f[base + src].lane.v : 0.0;
        break;
      }
      case BALLOT:
        L.ur = bal;
        break;
      case MFMA64:
      case MFMA32: {
        // A[i][k] from lane 16k + i, B[k][j] from lane 16k + j; output
        // register v of lane l: row (l/16 + 4v) in FP64, (4(l/16) + v) in
        // FP32; column l % 16
        const int c = l & 15, g = l >> 4;
        for (int v = 0; v < 4; ++v) {
          const int row = L.kind == MFMA64 ? g + 4 * v : 4 * g + v;
          double acc = L.acc[v];
          for (int k = 0; k < 4; ++k) {
            const int la = base + 16 * k + row, lb = base + 16 * k + c;
            const double a = la < end ? s.f[la].lane.a : 0.0;
            const double b = lb < end ? s.f[lb].lane.b : 0.0;
            acc += a * b;
          }
          L.racc[v] = L.kind == MFMA32 ? double(float(acc)) : acc;
        }
        break;
      }
      default:
        std::fprintf(stderr, "simt: unknown cross-lane operation\n");
        std::abort();
    }
    x.state = RUN;
  }
  return true;
}

// Run the workgroups `bids` (nt threads each) side by side to completion:
// a group of an ordinary launch, or the whole grid of a cooperative one,
// whose grid barrier spins with s_sleep (a yield here).
inline void run_blocks(const std::vector<int> &bids, int nt, int gdim,
                       const std::function<void()> &body) {
  Sched &s = S();
  const int nblk = (int)bids.size();
  constexpr size_t kStack = 1u << 20;
  const int total = nblk * nt;
  s.f.clear();
  s.f.resize(total);
  s.nt = nt;
  s.gdim = gdim;
  g_bdim = (unsigned)nt;
  g_gdim = (unsigned)gdim;
  s.body = &body;
  while ((int)s.stacks.size() < total) s.stacks.push_back(new char[kStack]);
  for (int t = 0; t < total; ++t) {
    Fiber &x = s.f[t];
    x.stack = s.stacks[t];
    // initial frame: six zero registers, then the entry point as the return
    // address, then a dummy return slot (16-byte alignment at entry)
    uintptr_t *sp = reinterpret_cast<uintptr_t *>(
        (reinterpret_cast<uintptr_t>(x.stack) + kStack) & ~uintptr_t(15));
    *--sp = 0;
    *--sp = reinterpret_cast<uintptr_t>(&fiber_entry);
    for (int r = 0; r < 6; ++r) *--sp = 0;
    x.sp = sp;
  }
  // per-workgroup LDS images when several workgroups run side by side
  const size_t lds_bytes = (__start_simt_lds && __stop_simt_lds)
                               ? size_t(__stop_simt_lds - __start_simt_lds) : 0;
  // LDS holds junk when a workgroup starts (as on the device, where it
  // keeps whatever the previous workgroup on that CU left): every byte is
  // set to 0xFF, a NaN in every float and double and -1 in every integer, so
  // a read before the workgroup's own write shows in the results
  std::vector<std::vector<char>> lds;
  int lds_loaded = 0;
  if (lds_bytes) std::memset(__start_simt_lds, 0xFF, lds_bytes);
  if (nblk > 1 && lds_bytes) lds.assign(nblk, std::vector<char>(lds_bytes, char(0xFF)));
  // sweeps alternate between ascending and descending thread order, so a
  // read that is not ordered after its write by a barrier sees the stale
  // value in one of the two orders; SIMT_SHUFFLE=<seed> takes a fresh
  // pseudo-random order each sweep instead (more orderings, reproducible):
  // the workgroups in a random order, each one's threads in a random order
  // (a workgroup's threads stay together, so its LDS image is swapped in
  // once per sweep)
  static const unsigned long long shuffle_seed = [] {
    const char *e = std::getenv("SIMT_SHUFFLE");
    return e ? std::strtoull(e, nullptr, 10) : 0ull;
  }();
  static unsigned long long rng = shuffle_seed * 6364136223846793005ull + 1442695040888963407ull;
  std::vector<int> order;
  if (shuffle_seed) {
    order.resize((size_t)total);
    for (int k = 0; k < total; ++k) order[(size_t)k] = k;
  }
  bool down = false;
  for (;;) {
    bool ran = false;
    down = !down;
    if (shuffle_seed) {
      // Fisher-Yates with a 64-bit LCG, over the workgroups and within each
      auto pick = [&](int k) {
        rng = rng * 6364136223846793005ull + 1442695040888963407ull;
        return (int)((rng >> 33) % (unsigned long long)(k + 1));
      };
      std::vector<int> blocks((size_t)nblk);
      for (int b = 0; b < nblk; ++b) blocks[(size_t)b] = b;
      for (int k = nblk - 1; k > 0; --k) std::swap(blocks[(size_t)k], blocks[(size_t)pick(k)]);
      size_t o = 0;
      for (int b : blocks) {
        const size_t b0 = o;
        for (int t = 0; t < nt; ++t) order[o++] = b * nt + t;
        for (int k = nt - 1; k > 0; --k) std::swap(order[b0 + (size_t)k], order[b0 + (size_t)pick(k)]);
      }
    }
    for (int k = 0; k < total; ++k) {
      const int t = shuffle_seed ? order[(size_t)k] : (down ? total - 1 - k : k);
      if (s.f[t].state != RUN) continue;
      ran = true;
      if (!lds.empty() && t / nt != lds_loaded) {
        std::memcpy(lds[lds_loaded].data(), __start_simt_lds, lds_bytes);
        lds_loaded = t / nt;
        std::memcpy(__start_simt_lds, lds[lds_loaded].data(), lds_bytes);
      }
      s.cur = t;
      s.bid = bids[t / nt];
      g_tid = (unsigned)(t % nt);
      g_bid = (unsigned)s.bid;
#ifdef SIMT_ASAN
      void *fake = nullptr;
      __sanitizer_start_switch_fiber(&fake, s.f[t].stack, kStack);
#endif
      simt_switch(&s.main_sp, s.f[t].sp);
#ifdef SIMT_ASAN
      __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
    }
    // cross-lane operations, then workgroup barriers, that can complete
    bool progress = false, all_done = true;
    for (int b = 0; b < nblk; ++b) {
      const int b0 = b * nt, b1 = b0 + nt;
      for (int w0 = b0; w0 < b1; w0 += kWaveLanes)
        progress |= resolve_wave(w0, std::min(b1, w0 + kWaveLanes));
      bool all_barrier = true, some_barrier = false, some_done = false;
      for (int t = b0; t < b1; ++t) {
        const State st = s.f[t].state;
        all_barrier &= st == BARRIER || st == DONE;
        some_barrier |= st == BARRIER;
        some_done |= st == DONE;
        all_done &= st == DONE;
      }
      if (all_barrier && some_barrier) {
        // a barrier reached by only part of the workgroup (others finished)
        // is a divergent barrier: report it
        if (some_done) {
          std::fprintf(stderr, "simt: barrier with finished threads (block %d)\n", bids[b]);
          std::abort();
        }
        for (int t = b0; t < b1; ++t) s.f[t].state = RUN;
        progress = true;
      }
    }
    if (all_done) break;
    if (!ran && !progress) {
      std::fprintf(stderr, "simt: deadlock (%d blocks from %d)\n", nblk, bids[0]);
      // where the threads wait: runs of equal (state, call site)
      static const char *names[] = {"run", "barrier", "cross-lane", "done"};
      for (int t = 0; t < total;) {
        int e = t + 1;
        while (e < total && s.f[e].state == s.f[t].state && s.f[e].lane.line == s.f[t].lane.line &&
               s.f[e].lane.file == s.f[t].lane.file)
          ++e;
        std::fprintf(stderr, "  threads %d-%d: %s at %s:%d\n", t, e - 1, names[s.f[t].state],
                     s.f[t].lane.file ? s.f[t].lane.file : "?", s.f[t].lane.line);
        t = e;
      }
      std::abort();
    }
  }
  s.cur = -1;
}

// yield from a spin-wait (other threads, also of other workgroups, run)
inline void spin_yield() {
  Sched &s = S();
  s.f[s.cur].state = RUN;
  yield_to_main();
}

// SIMT_WATCHDOG=<seconds>: a launch running longer prints where the
// current thread is and aborts (a thread spinning without yielding keeps
// the others from running)
inline void watchdog_handler(int) {
  char msg[96];
  const int k = std::snprintf(msg, sizeof msg, "simt: watchdog in block %u thread %u\n", g_bid, g_tid);
  (void)!write(2, msg, k);
  void *frames[48];
  const int nf = backtrace(frames, 48);
  backtrace_symbols_fd(frames, nf, 2);
  _exit(3);
}
inline void arm_watchdog() {
  static const int secs = [] {
    const char *e = std::getenv("SIMT_WATCHDOG");
    return e ? std::atoi(e) : 0;
  }();
  if (secs <= 0) return;
  signal(SIGALRM, watchdog_handler);
  alarm((unsigned)secs);
}

// workgroups of an ordinary launch that run side by side
inline int side_by_side() {
  static const int k = [] {
    const char *e = std::getenv("SIMT_SIDE_BY_SIDE");
    const int v = e ? std::atoi(e) : 4;
    return v < 1 ? 1 : v;
  }();
  return k;
}

template <class F>
inline void launch(dim3 grid, dim3 block, F &&kernel_call) {
  arm_watchdog();
  const std::function<void()> body = [&]() { kernel_call(); };
  // blocks alternately from the top and the bottom of the grid
  const int g = (int)grid.x;
  std::vector<int> order;
  for (int lo = 0, hi = g - 1; lo <= hi; ++lo, --hi) {
    order.push_back(hi);
    if (lo != hi) order.push_back(lo);
  }
  const int k = side_by_side();
  for (size_t i = 0; i < order.size(); i += (size_t)k) {
    const std::vector<int> ids(order.begin() + (long)i,
                               order.begin() + (long)std::min(order.size(), i + (size_t)k));
    run_blocks(ids, (int)block.x, g, body);
  }
  if (std::getenv("SIMT_WATCHDOG")) alarm(0);
}

template <class F>
inline void launch_cooperative(dim3 grid, dim3 block, F &&kernel_call) {
  arm_watchdog();
  const std::function<void()> body = [&]() { kernel_call(); };
  std::vector<int> ids((size_t)grid.x);
  for (int b = 0; b < (int)grid.x; ++b) ids[(size_t)b] = b;
  run_blocks(ids, (int)block.x, (int)grid.x, body);
  if (std::getenv("SIMT_WATCHDOG")) alarm(0);
}

// Resource usage of each kernel as the gfx950 build reports it (registered
// by the host build): registers per lane and static LDS per workgroup.
struct KernelRes {
  const void *fn;
  int vgpr, agpr, lds;
};
inline std::vector<KernelRes> &kernel_resources() {
  static std::vector<KernelRes> r;
  return r;
}
inline bool register_resources(const void *fn, int vgpr, int agpr, int lds) {
  kernel_resources().push_back({fn, vgpr, agpr, lds});
  return true;
}
inline const KernelRes &resources_of(const void *fn) {
  for (const KernelRes &k : kernel_resources())
    if (k.fn == fn) return k;
  std::fprintf(stderr, "simt: no resource record for a kernel\n");
  std::abort();
}

inline Lane &me() { return S().f[S().cur].lane; }

}  // namespace simt

inline const ::simt::DimRef threadIdx{::simt::g_tid, 0u, 0u};
inline const ::simt::DimRef blockIdx{::simt::g_bid, 0u, 0u};
inline const ::simt::DimRef blockDim{::simt::g_bdim, 1u, 1u};
inline const ::simt::DimRef gridDim{::simt::g_gdim, 1u, 1u};

inline void __syncthreads(const char *file = __builtin_FILE(), int line = __builtin_LINE()) {
  ::simt::Lane &L = ::simt::me();
  L.file = file; L.line = line;
  ::simt::wait(::simt::BARRIER);
}
inline void __threadfence() {}

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64, const char *file = __builtin_FILE(),
                    int line = __builtin_LINE()) {
  ::simt::Lane &L = ::simt::me();
  L.kind = ::simt::SHFL_XOR; L.arg = mask; L.width = width; L.v = double(v);
  L.file = file; L.line = line;
  ::simt::wait(::simt::WAVE);
  return T(L.r);
}
template <class T>
inline T __shfl(T v, int src, int width = 64, const char *file = __builtin_FILE(),
                int line = __builtin_LINE()) {
  ::simt::Lane &L = ::simt::me();
  L.kind = ::simt::SHFL; L.arg = src; L.width = width; L.v = double(v);
  L.file = file; L.line = line;
  ::simt::wait(::simt::WAVE);
  return T(L.r);
}
inline unsigned long long __ballot(int pred, const char *file = __builtin_FILE(),
                                   int line = __builtin_LINE()) {
  ::simt::Lane &L = ::simt::me();
  L.kind = ::simt::BALLOT; L.pred = pred != 0; L.width = 64;
  L.file = file; L.line = line;
  ::simt::wait(::simt::WAVE);
  return L.ur;
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }

template <class V>
inline V simt_mfma(double a, double b, V c, int kind, const char *file = __builtin_FILE(),
                   int line = __builtin_LINE()) {
  ::simt::Lane &L = ::simt::me();
  L.kind = kind; L.a = a; L.b = b; L.width = 64;
  L.file = file; L.line = line;
  for (int v = 0; v < 4; ++v) L.acc[v] = double(c[v]);
  ::simt::wait(::simt::WAVE);
  V r;
  for (int v = 0; v < 4; ++v) r[v] = (decltype(c[0] + 0))L.racc[v];
  return r;
}
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) \
  simt_mfma((double)(a), (double)(b), (c), ::simt::MFMA64)
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) \
  simt_mfma((double)(a), (double)(b), (c), ::simt::MFMA32)
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_s_sleep(x) ::simt::spin_yield()

inline unsigned long long wall_clock64() { return ++::simt::S().clock; }

// atomics: fibers of one workgroup run on one host thread, one at a time
template <class T>
inline T atomicAdd(T *p, T v) { T o = *p; *p = o + v; return o; }
template <class T>
inline T atomicOr(T *p, T v) { T o = *p; *p = o | v; return o; }
template <class T>
inline T simt_atomic_load(T *p) { return *p; }
template <class T, class V>
inline void simt_atomic_store(T *p, V v) { *p = T(v); }
template <class T, class V>
inline T simt_atomic_fetch_add(T *p, V v) { T o = *p; *p = T(o + v); return o; }
#define __hip_atomic_load(p, order, scope) simt_atomic_load(p)
#define __hip_atomic_store(p, v, order, scope) simt_atomic_store(p, v)
#define __hip_atomic_fetch_add(p, v, order, scope) simt_atomic_fetch_add(p, v)

// ---- runtime API -------------------------------------------------------------
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotSupported = 801, hipErrorInvalidValue = 1 };
typedef struct simt_stream *hipStream_t;
typedef struct simt_event { double t; } *hipEvent_t;
typedef struct simt_graph *hipGraph_t;
typedef struct simt_graph_exec *hipGraphExec_t;
typedef struct simt_graph_node *hipGraphNode_t;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipStreamNonBlocking = 1 };
enum hipDeviceAttribute_t { hipDeviceAttributeWallClockRate = 1 };

struct hipDeviceProp_t {
  int multiProcessorCount;
  size_t sharedMemPerBlock;
  size_t maxSharedMemoryPerMultiProcessor;
};
struct hipFuncAttributes { size_t sharedSizeBytes; };
struct hipKernelNodeParams {
  void *func; dim3 gridDim; dim3 blockDim; void **kernelParams; void **extra;
  unsigned sharedMemBytes;
};

// compute units of the emulated device (gfx950: 256)
#ifndef SIMT_CU_COUNT
#define SIMT_CU_COUNT 256
#endif

inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
// SIMT_CUS (environment) overrides the build-time count, for the runs of a
// cooperative launch, whose whole grid (one workgroup per CU) runs side by side
inline int simt_cu_count() {
  static const int n = [] {
    const char *e = std::getenv("SIMT_CUS");
    const int v = e ? std::atoi(e) : 0;
    return v > 0 ? v : SIMT_CU_COUNT;
  }();
  return n;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
  p->multiProcessorCount = simt_cu_count();
  p->sharedMemPerBlock = 160 * 1024;
  p->maxSharedMemoryPerMultiProcessor = 160 * 1024;
  return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) { *v = 100000; return hipSuccess; }
inline hipError_t hipFuncGetAttributes(hipFuncAttributes *a, const void *fn) {
  a->sharedSizeBytes = (size_t)::simt::resources_of(fn).lds;
  return hipSuccess;
}
// Workgroups of `block` threads one CU holds at once, from the kernel's
// registers and LDS: four SIMDs, each with 512 registers per lane shared by
// its waves (allocated in granules of 8, vector then accumulation registers)
// and at most 8 waves; a workgroup's waves spread over the four SIMDs;
// 160 KiB of LDS per CU.
template <class F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, F fn, int block, size_t dyn) {
  const ::simt::KernelRes &r = ::simt::resources_of((const void *)fn);
  const int regs = ((r.vgpr + 7) / 8) * 8 + ((r.agpr + 7) / 8) * 8;
  const int waves_simd = std::min(8, regs > 0 ? 512 / regs : 8);
  const int waves = (block + 63) / 64, per_simd = (waves + 3) / 4;
  int wg = per_simd > 0 ? waves_simd / per_simd : 0;
  const size_t lds = (size_t)r.lds + dyn;
  if (lds > 0) wg = std::min(wg, (int)((160u * 1024u) / lds));
  *n = std::max(0, wg);
  return hipSuccess;
}
inline hipError_t hipMalloc(void **p, size_t bytes) {
  *p = std::malloc(bytes ? bytes : 1);
  if (*p) std::memset(*p, 0xFF, bytes);   // device memory starts with junk (NaN, -1)
  return *p ? hipSuccess : hipErrorInvalidValue;
}
template <class T>
inline hipError_t hipMalloc(T **p, size_t bytes) { return hipMalloc((void **)p, bytes); }
// one array of the device arena (kept until the process ends)
inline void *simt_array_alloc(size_t bytes) {
  const size_t b = (bytes + 15) & ~size_t(15);
  void *p = std::malloc(b ? b : 16);
  if (p) std::memset(p, 0xFF, b ? b : 16);
  return p;
}
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new char(0));
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { delete reinterpret_cast<char *>(s); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
// launches run to completion when they are issued
inline hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
inline double simt_now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new simt_event{0.0}; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t = nullptr) { e->t = simt_now_ms(); return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  *ms = float(b->t - a->t);
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
// Graphs of kernel nodes (and cooperative launches), replayed in the order the nodes were added (each
// node depends on the one before it where the library builds them).  A
// kernel reaches a node through a binder registered for its address, which
// copies the argument values when the node is added, as the runtime does.
namespace simt {
using Binder = std::function<std::function<void()>(void **)>;
inline std::vector<std::pair<const void *, Binder>> &kernel_binders() {
  static std::vector<std::pair<const void *, Binder>> r;
  return r;
}
inline bool register_kernel(const void *fn, Binder b) {
  kernel_binders().push_back({fn, std::move(b)});
  return true;
}
struct GraphNode {
  std::function<void()> call;
  dim3 grid, block;
};
}  // namespace simt
struct simt_graph { std::vector<::simt::GraphNode> nodes; };
struct simt_graph_exec { std::vector<::simt::GraphNode> nodes; };
struct simt_graph_node { int index; };
// cooperative launch: the whole grid side by side
inline hipError_t hipLaunchCooperativeKernel(const void *fn, dim3 grid, dim3 block, void **args,
                                             size_t, hipStream_t) {
  for (auto &kb : ::simt::kernel_binders())
    if (kb.first == fn) {
      const std::function<void()> call = kb.second(args);
      ::simt::launch_cooperative(grid, block, call);
      return hipSuccess;
    }
  return hipErrorNotSupported;
}
inline hipError_t hipGraphCreate(hipGraph_t *g, unsigned) { *g = new simt_graph; return hipSuccess; }
inline hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t g, const hipGraphNode_t *,
                                        size_t, const hipKernelNodeParams *p) {
  for (auto &kb : ::simt::kernel_binders())
    if (kb.first == p->func) {
      g->nodes.push_back({kb.second(p->kernelParams), p->gridDim, p->blockDim});
      static simt_graph_node dummy{0};
      *node = &dummy;
      return hipSuccess;
    }
  return hipErrorNotSupported;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  *e = new simt_graph_exec{g->nodes};
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto &nd : e->nodes) ::simt::launch(nd.grid, nd.block, nd.call);
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
