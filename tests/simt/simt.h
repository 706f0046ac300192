// CPU execution of HIP kernel source (test infrastructure): every GPU thread of a block is
// a fiber on one OS thread (x86-64 context switch below), several blocks run at once on OS
// threads of their own (so `__shared__` = static thread_local is per block), barriers and
// wave intrinsics switch fibers.  Built with -fsanitize=address it catches out-of-range
// accesses in the real kernel text; threads of a block that finish while others of the
// same block wait at a barrier (a block-divergent exit) abort the run with a message.
#pragma once
#include <sanitizer/common_interface_defs.h>
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <type_traits>
#include <vector>

struct SimDim3 { uint32_t x = 1, y = 1, z = 1; };
inline thread_local SimDim3 threadIdx, blockIdx;
inline SimDim3 blockDim, gridDim;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __align__(x) alignas(x)

namespace simt {
extern "C" void simt_switch(void** from_sp, void* to_sp);
asm(R"(
.text
.globl simt_switch
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
)");
struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  bool done = false;
  uint32_t tid = 0;
  int waiting = 0;  // 1 block barrier, 2 wave barrier
};
inline thread_local void* sched_sp = nullptr;
inline thread_local const void* sched_bottom = nullptr;
inline thread_local size_t sched_size = 0;
// (the stacks go with the OS thread that ran the fibers)
struct Fibers : std::vector<Fiber> {
  ~Fibers() {
    for (auto& f : *this) std::free(f.stack);
  }
};
inline thread_local Fibers fibers;
inline thread_local int cur = 0;
inline std::function<void()>* body = nullptr;  // shared by the block threads (read only)
inline thread_local uint64_t bar_gen = 0;
inline thread_local uint32_t bar_count = 0;
inline thread_local uint64_t wbar_gen[16];
inline thread_local uint32_t wbar_count[16];
inline thread_local uint64_t xch[16][64];
inline thread_local uint64_t switches = 0;
#ifndef SIMT_STACK
#define SIMT_STACK (256 * 1024)
#endif
constexpr size_t kStack = SIMT_STACK;

inline void to_sched() {
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, sched_bottom, sched_size);
  simt_switch(&fibers[cur].sp, sched_sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}
inline void yield() {
  ++switches;
  to_sched();
}
inline int wave_of() { return (int)(threadIdx.x / 64); }
inline int lane_of() { return (int)(threadIdx.x % 64); }
inline uint32_t wave_lanes(int w) { return std::min<uint32_t>(64, blockDim.x - 64 * (uint32_t)w); }
inline void block_sync() {
  const uint64_t g = bar_gen;
  if (++bar_count == blockDim.x) {
    bar_count = 0;
    ++bar_gen;
    return;
  }
  fibers[cur].waiting = 1;
  while (bar_gen == g) yield();
  fibers[cur].waiting = 0;
}
inline void wave_sync() {
  const int w = wave_of();
  const uint64_t g = wbar_gen[w];
  if (++wbar_count[w] == wave_lanes(w)) {
    wbar_count[w] = 0;
    ++wbar_gen[w];
    return;
  }
  fibers[cur].waiting = 2;
  while (wbar_gen[w] == g) yield();
  fibers[cur].waiting = 0;
}
template <typename T> inline uint64_t bits(T v) { uint64_t b = 0; std::memcpy(&b, &v, sizeof(T)); return b; }
template <typename T> inline T unbits(uint64_t b) { T v; std::memcpy(&v, &b, sizeof(T)); return v; }
template <typename T> inline T exch(T v, int src) {
  static_assert(sizeof(T) <= 8, "");
  const int w = wave_of();
  xch[w][lane_of()] = bits(v);
  wave_sync();
  const T r = (src >= 0 && src < (int)wave_lanes(w)) ? unbits<T>(xch[w][src]) : v;
  wave_sync();
  return r;
}
inline void trampoline() {
  __sanitizer_finish_switch_fiber(nullptr, &sched_bottom, &sched_size);
  (*body)();
  fibers[cur].done = true;
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(nullptr, sched_bottom, sched_size);  // this fiber ends
  (void)fake;
  simt_switch(&fibers[cur].sp, sched_sp);
  std::abort();  // a finished fiber is never resumed
}
// One block on the calling OS thread: its threads as fibers.
inline void run_block(uint32_t b, uint32_t block) {
  if (fibers.size() < block) fibers.resize(block);
  for (auto& f : fibers)
    if (!f.stack) f.stack = (char*)std::malloc(kStack);
  blockIdx = {b, 0, 0};
  bar_gen = bar_count = 0;
  std::memset(wbar_gen, 0, sizeof(wbar_gen));
  std::memset(wbar_count, 0, sizeof(wbar_count));
  for (uint32_t t = 0; t < block; ++t) {
    Fiber& f = fibers[t];
    f.done = false;
    f.tid = t;
    f.waiting = 0;
    // initial frame: six callee-saved registers, then the entry as the return address
    uintptr_t top = ((uintptr_t)f.stack + kStack) & ~(uintptr_t)15;
    void** sp = (void**)top;
    *--sp = nullptr;                  // alignment slot (entry sees rsp = 8 mod 16)
    *--sp = (void*)&trampoline;       // popped by `ret`
    for (int r = 0; r < 6; ++r) *--sp = nullptr;
    f.sp = sp;
  }
  uint32_t alive = block;
  while (alive) {
    uint32_t progressed = 0;
    alive = 0;
    for (uint32_t t = 0; t < block; ++t) {
      Fiber& f = fibers[t];
      if (f.done) continue;
      cur = (int)t;
      threadIdx = {t, 0, 0};
      const uint64_t g0 = bar_gen;
      void* fake = nullptr;
      __sanitizer_start_switch_fiber(&fake, f.stack, kStack);
      simt_switch(&sched_sp, f.sp);
      __sanitizer_finish_switch_fiber(fake, &sched_bottom, &sched_size);
      if (f.done || bar_gen != g0) ++progressed;
      if (!f.done) ++alive;
    }
    if (alive && !progressed) {
      bool all_wait = true;
      uint32_t done_n = 0;
      for (uint32_t t = 0; t < block; ++t) {
        if (!fibers[t].done && fibers[t].waiting == 0) all_wait = false;
        done_n += fibers[t].done ? 1 : 0;
      }
      if (all_wait && done_n > 0) {
        fprintf(stderr, "simt: block %u: %u threads finished while others wait at a barrier\n", b, done_n);
        std::abort();
      }
    }
  }
}
// Run `kern()` on grid x block threads: `workers` OS threads take blocks from a shared
// counter, so that up to `workers` blocks run at once (each with its own LDS).
template <typename F>
void launch(uint32_t grid, uint32_t block, F kern, unsigned workers = 1) {
  gridDim = {grid, 1, 1};
  blockDim = {block, 1, 1};
  std::function<void()> fn = kern;
  body = &fn;
  std::atomic<uint32_t> next{0};
  auto worker = [&] {
    for (;;) {
      const uint32_t b = next.fetch_add(1);
      if (b >= grid) break;
      run_block(b, block);
    }
  };
  if (workers <= 1) {
    worker();
  } else {
    std::vector<std::thread> th;
    for (unsigned i = 0; i < workers; ++i) th.emplace_back(worker);
    for (auto& t : th) t.join();
  }
  body = nullptr;
}
}  // namespace simt

inline void __syncthreads() { simt::block_sync(); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_block() {}
template <typename T> inline T __shfl_up(T v, unsigned d, int = 64) { return simt::exch(v, simt::lane_of() - (int)d); }
template <typename T> inline T __shfl_down(T v, unsigned d, int = 64) { return simt::exch(v, simt::lane_of() + (int)d); }
template <typename T> inline T __shfl_xor(T v, int m, int = 64) { return simt::exch(v, simt::lane_of() ^ m); }
template <typename T> inline T __shfl(T v, int src, int = 64) { return simt::exch(v, src); }
inline uint64_t __builtin_amdgcn_ballot_w64(bool p) {
  const int w = simt::wave_of();
  simt::xch[w][simt::lane_of()] = p ? 1 : 0;
  simt::wave_sync();
  uint64_t m = 0;
  for (uint32_t l = 0; l < simt::wave_lanes(w); ++l) if (simt::xch[w][l]) m |= 1ull << l;
  simt::wave_sync();
  return m;
}
template <typename T> inline T __builtin_amdgcn_readfirstlane(T v) { return simt::exch(v, 0); }
// DPP quad permutation (controls below 0x100: lane 4q + i reads lane 4q + ctrl[2i+1:2i])
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int, int, bool) {
  if (ctrl < 0 || ctrl > 0xFF) std::abort();  // only quad_perm is emulated
  (void)old;
  const int lane = simt::lane_of();
  return simt::exch(src, (lane & ~3) | ((ctrl >> (2 * (lane & 3))) & 3));
}
// ds_swizzle in its bit mode (offset bit 15 clear): within each 32 lanes, lane i reads
// ((i & and) | or) ^ xor
inline int __builtin_amdgcn_ds_swizzle(int v, int pattern) {
  if (pattern & 0x8000) std::abort();  // only the bit mode is emulated
  const int lane = simt::lane_of();
  const int am = pattern & 0x1F, om = (pattern >> 5) & 0x1F, xm = (pattern >> 10) & 0x1F;
  return simt::exch(v, (lane & 32) | (((lane & 31 & am) | om) ^ xm));
}
inline void __builtin_amdgcn_wave_barrier() {}
inline void __builtin_amdgcn_s_sleep(int) {}
inline int __popc(uint32_t v) { return __builtin_popcount(v); }
inline int __popcll(uint64_t v) { return __builtin_popcountll(v); }
inline int __ffs(uint32_t v) { return __builtin_ffs(v); }
inline int __ffsll(uint64_t v) { return __builtin_ffsll(v); }
inline int __clz(uint32_t v) { return v ? __builtin_clz(v) : 32; }
inline int __clzll(uint64_t v) { return v ? __builtin_clzll(v) : 64; }
template <typename T> inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <typename T> inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <typename T> inline T atomicAnd(T* p, T v) { return __atomic_fetch_and(p, v, __ATOMIC_SEQ_CST); }
template <typename T> inline T atomicMin(T* p, T v) { T o = __atomic_load_n(p, __ATOMIC_SEQ_CST); while (v < o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {} return o; }
template <typename T> inline T atomicMax(T* p, T v) { T o = __atomic_load_n(p, __ATOMIC_SEQ_CST); while (v > o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {} return o; }
template <typename T> inline T atomicExch(T* p, T v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
template <typename T, typename U> inline auto min(T a, U b) -> typename std::common_type<T, U>::type { return a < b ? a : b; }
template <typename T, typename U> inline auto max(T a, U b) -> typename std::common_type<T, U>::type { return a > b ? a : b; }
template <typename T> inline T min(T a, T b) { return a < b ? a : b; }
template <typename T> inline T max(T a, T b) { return a > b ? a : b; }
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef int hipError_t;
