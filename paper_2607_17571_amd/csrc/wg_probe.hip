// Synchronisation costs behind the loop-policy ablation (Section V-B): what a grid-wide
// barrier inside one persistent, cooperative launch costs on this device, against a
// kernel boundary (the next launch on the same in-order stream), which is what the
// engine's multi-block iterations pay between stages.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wg.h"

namespace {

constexpr uint32_t kProbeThreads = 256;
constexpr uint32_t kProbeSpinLimit = 1u << 20;  // polls of one wait before it gives up
constexpr uint32_t kProbeLaunchesMax = 512;     // empty launches timed (queued ahead of time)
constexpr uint64_t kProbeDelayUs = 20000;        // delay ahead of the timed launches

// `rounds` grid-wide barriers.  state[0] counts the arrivals of the current round at the
// top level, GEN is the round's generation, FAIL is set by a wait that gave up (every block
// then leaves at its next barrier, so the launch always drains); each word that blocks
// update or poll has a line of its own, so polls do not contend with arrivals.  Flat (GROUPS
// 1): every block arrives on state[0].  Two-level (GROUPS 8, the device's XCDs, to which
// consecutive blocks are dealt in turn): a block arrives on its group's counter (each on a
// line of its own), and the last of each group arrives on state[0].  The last arrival at
// the top resets the count and then advances the generation (release), which the waiting
// blocks poll (acquire); each group's last block resets its group counter before arriving
// at the top, so every reset is visible before any block counts itself into the next round.
constexpr uint32_t kProbeLine = 64;  // u32 words between counters
constexpr uint32_t kProbeGen = kProbeLine * 9, kProbeFail = kProbeLine * 10;
constexpr size_t kProbeStateBytes = kProbeLine * 11 * sizeof(uint32_t);
template <uint32_t GROUPS>
__global__ __launch_bounds__(kProbeThreads) void k_grid_barrier_probe(uint32_t* state, uint32_t rounds) {
  __shared__ int s_stop;
  const uint32_t groups = GROUPS < gridDim.x ? GROUPS : gridDim.x;
  const uint32_t g = blockIdx.x % groups;
  const uint32_t gsize = gridDim.x / groups + (g < gridDim.x % groups ? 1u : 0u);
  uint32_t* const gcount = state + kProbeLine * (g + 1);
  for (uint32_t r = 0; r < rounds; ++r) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int stop = 0;
      const uint32_t gen = __hip_atomic_load(&state[kProbeGen], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      bool top = true;  // this block arrives at the top level
      if (groups > 1) {
        top = __hip_atomic_fetch_add(gcount, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1;
        if (top) __hip_atomic_store(gcount, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const bool last =
          top && __hip_atomic_fetch_add(&state[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == groups - 1;
      if (last) {
        __hip_atomic_store(&state[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&state[kProbeGen], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t spins = 0;
        while (__hip_atomic_load(&state[kProbeGen], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          if (++spins > kProbeSpinLimit) {
            __hip_atomic_fetch_or(&state[kProbeFail], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (__hip_atomic_load(&state[kProbeFail], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) stop = 1;
      s_stop = stop;
    }
    __syncthreads();
    if (s_stop) return;
  }
}

// The same `rounds` barriers through the runtime's own grid synchronisation for cooperative
// launches (cooperative groups).
__global__ __launch_bounds__(kProbeThreads) void k_grid_sync_probe(uint32_t* state, uint32_t rounds) {
  (void)state;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (uint32_t r = 0; r < rounds; ++r) grid.sync();
}

__global__ __launch_bounds__(kProbeThreads) void k_empty_probe(uint32_t* state) { (void)state; }

// Holds the stream for `ticks` of the constant real-time clock (bounded by construction), so
// that the launches queued behind it are all in the queue before the timed window opens and
// the window measures the device, not the host's launch rate.
__global__ __launch_bounds__(kProbeThreads) void k_delay_probe(uint64_t ticks) {
  if (threadIdx.x != 0) return;
  const uint64_t t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

// The caller's current device, made current again when the call returns.
struct DeviceRestore {
  int prev = -1;
  DeviceRestore() {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  }
  ~DeviceRestore() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

struct ProbeRes {
  hipStream_t s = nullptr;
  hipEvent_t ev[6] = {};
  uint32_t* state = nullptr;
  ~ProbeRes() {
    if (state) (void)hipFree(state);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (s) (void)hipStreamDestroy(s);
  }
};

}  // namespace

extern "C" wg_status wg_probe_sync_costs(int device, uint32_t blocks, uint32_t rounds, double* barrier_us,
                                          double* barrier2_us, double* barrier_cg_us, double* launch_us) {
  if (!barrier_us || !barrier2_us || !barrier_cg_us || !launch_us || blocks == 0 || blocks > 2048 || rounds == 0 || rounds > 1000000)
    return WG_ERR_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return WG_ERR_INVALID_ARG;
  const DeviceRestore restore;  // (destroyed last: after the probe's resources are freed)
  if (hipSetDevice(device) != hipSuccess) return WG_ERR_DEVICE;
  int coop = 0, cus = 0, per_cu = 0, clock_khz = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop ||
      hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || clock_khz <= 0 ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_grid_barrier_probe<1>, (int)kProbeThreads, 0) !=
          hipSuccess)
    return WG_ERR_DEVICE;
  // every block of a barrier launch must be resident at once
  if ((uint64_t)per_cu * (uint64_t)cus < blocks) return WG_ERR_INVALID_ARG;
  ProbeRes p;
  if (hipStreamCreateWithFlags(&p.s, hipStreamNonBlocking) != hipSuccess) return WG_ERR_DEVICE;
  for (hipEvent_t& e : p.ev)
    if (hipEventCreate(&e) != hipSuccess) return WG_ERR_DEVICE;
  if (hipMalloc(&p.state, kProbeStateBytes) != hipSuccess) return WG_ERR_OUT_OF_MEMORY;
  // kind 0: flat, 1: two-level, 2: the runtime's grid synchronisation
  auto barriers = [&](int kind, uint32_t r, hipEvent_t a, hipEvent_t b) -> bool {
    if (hipMemsetAsync(p.state, 0, kProbeStateBytes, p.s) != hipSuccess) return false;
    void* args[] = {&p.state, &r};
    if (a && hipEventRecord(a, p.s) != hipSuccess) return false;
    const void* k = kind == 0   ? (const void*)k_grid_barrier_probe<1>
                    : kind == 1 ? (const void*)k_grid_barrier_probe<8>
                                : (const void*)k_grid_sync_probe;
    if (hipLaunchCooperativeKernel(k, dim3(blocks), dim3(kProbeThreads), args, 0, p.s) != hipSuccess) return false;
    return !b || hipEventRecord(b, p.s) == hipSuccess;
  };
  uint32_t failed = 0;
  // per kind: a warm-up, then one launch without barriers and one with `rounds` of them
  float tb[3] = {0, 0, 0};
  for (int kind = 0; kind < 3; ++kind) {
    if (!barriers(kind, 1, nullptr, nullptr) || !barriers(kind, 0, p.ev[0], p.ev[1]) ||
        !barriers(kind, rounds, p.ev[2], p.ev[3]))
      return WG_ERR_DEVICE;
    if (hipMemcpyAsync(&failed, p.state + kProbeFail, sizeof(uint32_t), hipMemcpyDeviceToHost, p.s) != hipSuccess ||
        hipStreamSynchronize(p.s) != hipSuccess || failed != 0)
      return WG_ERR_DEVICE;
    float t0 = 0, t1 = 0;
    if (hipEventElapsedTime(&t0, p.ev[0], p.ev[1]) != hipSuccess ||
        hipEventElapsedTime(&t1, p.ev[2], p.ev[3]) != hipSuccess)
      return WG_ERR_DEVICE;
    tb[kind] = t1 - t0;
  }
  // dependent launches of an empty kernel of the same shape (up to kProbeLaunchesMax),
  // queued behind a delay so that the host's launch rate does not enter the window
  const uint32_t nl = rounds < kProbeLaunchesMax ? rounds : kProbeLaunchesMax;
  hipLaunchKernelGGL(k_empty_probe, dim3(blocks), dim3(kProbeThreads), 0, p.s, p.state);
  const uint64_t delay_ticks = kProbeDelayUs * (uint64_t)clock_khz / 1000;  // (the real-time clock's rate)
  hipLaunchKernelGGL(k_delay_probe, dim3(1), dim3(kProbeThreads), 0, p.s, delay_ticks);
  if (hipEventRecord(p.ev[4], p.s) != hipSuccess) return WG_ERR_DEVICE;
  for (uint32_t r = 0; r < nl; ++r) hipLaunchKernelGGL(k_empty_probe, dim3(blocks), dim3(kProbeThreads), 0, p.s, p.state);
  if (hipEventRecord(p.ev[5], p.s) != hipSuccess || hipGetLastError() != hipSuccess ||
      hipStreamSynchronize(p.s) != hipSuccess)
    return WG_ERR_DEVICE;
  float t2 = 0;
  if (hipEventElapsedTime(&t2, p.ev[4], p.ev[5]) != hipSuccess) return WG_ERR_DEVICE;
  *barrier_us = 1000.0 * (double)tb[0] / rounds;
  *barrier2_us = 1000.0 * (double)tb[1] / rounds;
  *barrier_cg_us = 1000.0 * (double)tb[2] / rounds;
  *launch_us = 1000.0 * (double)t2 / nl;
  return WG_OK;
}
