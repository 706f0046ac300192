// Device-side building blocks shared by the fixpoint kernels (gfx950, wave64).
//
// Relations are arrays of packed keys  key = inst << 2w | src << w | dst  where w is
// the radix field width (16, 24 or 32) chosen from the largest vertex id (Section V-C,
// adaptive bit-width selection).  With src in the high bits the numeric key order is the
// lexicographic (src, dst) order the pipeline keeps at every stage boundary (Section
// IV-A).  `inst` is non-zero only for batched solves.  A 32-bit key type is used when
// the key fits, which halves the bytes every stage streams.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wg {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// Control block: every size that decides a launch lives here, in device memory.
// Kernels read it at entry; the host reads it only at batch boundaries.
// ---------------------------------------------------------------------------
struct Ctrl {
  uint64_t D;            // |Delta^{i-1}|, input of the next join
  uint64_t F;            // |Full|
  uint64_t C;            // join candidates of the running iteration (saturating)
  uint64_t N;            // |Delta^i| produced by the running iteration
  uint64_t m_in;         // input edge count (prepare)
  uint64_t m_unique;     // |E| after sort + dedup
  uint64_t nu;           // distinct (inst, src) rows of the edge index
  uint64_t total_cand;   // candidates summed over completed iterations
  uint64_t cand_cap;     // capacity of each candidate buffer (keys)
  uint64_t full_cap;     // capacity of each Full buffer (keys)
  uint64_t delta_cap;    // capacity of each delta buffer (keys)
  uint64_t dsz_cap;      // capacity of the per-iteration delta-size array
  uint32_t iter;         // completed iterations
  uint32_t max_iter;     // 0: unlimited
  uint32_t done;         // the last delta was empty: fixpoint reached
  uint32_t overflow;     // bit 0 candidates, bit 1 Full, bit 2 delta, bit 3 size array
  uint32_t error;        // bit 0: a bounded device wait expired
  uint32_t limit_hit;    // max_iter reached with a non-empty delta
  uint32_t full_side;    // which Full buffer holds the current relation
  uint32_t delta_side;   // which delta buffer holds Delta^{i-1}
  uint32_t maxid;        // largest vertex id of the input
  uint32_t force_overflow_at;  // test hook: report a candidate overflow at this iteration
  uint32_t pad0;
  uint64_t D0;           // |Delta^0|, the seed size
  uint64_t total;        // hand-over of a launch-wide total to the launch's last claimer
};

// A halted loop turns every later kernel of the batch into a no-op.
__device__ __forceinline__ bool halted(const Ctrl* c) {
  return (c->done | c->overflow | c->error | c->limit_hit) != 0;
}

// ---------------------------------------------------------------------------
// Decoupled lookback state (single-pass scans, Section IV-B).
//
// A status word is  [63:62] flag | [61:40] epoch | [39:0] value.  flag 1 = tile
// aggregate, 2 = inclusive prefix.  Words from earlier launches carry another epoch and
// read as "not ready", so the status array never needs clearing between launches.  The
// block that makes a launch's last tile claim resets the counter and advances the epoch.
// ---------------------------------------------------------------------------
constexpr int kClaimLanes = 8;
struct LbState {
  uint32_t lane_ctr[kClaimLanes][64];  // one claim counter per 256-byte line
  uint32_t lanes_done;
  uint32_t epoch;
  uint32_t pad[62];
};

constexpr uint64_t kValMask = (1ull << 40) - 1;
constexpr uint32_t kEpochMask = (1u << 22) - 1;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint32_t launch_epoch(const LbState* st) {
  const uint32_t cur = __hip_atomic_load(const_cast<uint32_t*>(&st->epoch), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t e = (cur & kEpochMask) + 1;
  return e > kEpochMask ? 1u : e;
}

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  return s > kValMask ? kValMask : s;
}

__device__ __forceinline__ uint64_t status_word(uint64_t flag, uint32_t epoch, uint64_t v) {
  return flag | ((uint64_t)epoch << 40) | (v > kValMask ? kValMask : v);
}

__device__ __forceinline__ void status_store(uint64_t* p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Dynamic tile claims.  A tile only ever waits on tiles claimed before it in its own
// claim order, by blocks that are already running, so lookback cannot deadlock.  Claims
// go through 8 independent counters ("lanes", one per 256-byte line): block b draws from
// lane b % 8, whose k-th claim is tile 8k + lane.  Same-address atomics serialise at a
// few tens of ns each across the XCDs, so spreading them over 8 addresses keeps claims
// off the critical path.  The smallest unfinished tile is always either held by a running
// block or the next tile of its lane, which a block of that lane (all of whose earlier
// tiles are finished) claims next: progress is guaranteed.
//
// Every block ends with exactly one failing claim.  The last failing claim on a lane
// resets that lane; the last lane to finish (a second counter) marks the block that
// knows every block of the launch is done: it advances the epoch and may publish
// launch-wide results.
struct TileClaim {
  uint32_t tile;   // valid when `ok`
  bool ok;         // a tile was claimed
  bool last;       // this block closed the launch
};

__device__ __forceinline__ uint32_t lane_tiles(uint64_t ntiles, uint32_t lane) {
  return ntiles > lane ? (uint32_t)((ntiles - lane + kClaimLanes - 1) / kClaimLanes) : 0u;
}

__device__ __forceinline__ uint32_t lane_blocks(uint32_t lane) {
  return (gridDim.x - lane + kClaimLanes - 1) / kClaimLanes;
}

__device__ __forceinline__ TileClaim claim_tile(LbState* st, uint64_t ntiles, uint32_t* s_buf) {
  const uint32_t lane = blockIdx.x & (kClaimLanes - 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t k = atomicAdd(&st->lane_ctr[lane][0], 1u);
    uint32_t last = 0;
    const uint32_t tiles = lane_tiles(ntiles, lane);
    if (k >= tiles && k == tiles + lane_blocks(lane) - 1) {
      // final claim on this lane: reset it, then count finished lanes
      __hip_atomic_store(&st->lane_ctr[lane][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t lanes = gridDim.x < (uint32_t)kClaimLanes ? gridDim.x : (uint32_t)kClaimLanes;
      last = (atomicAdd(&st->lanes_done, 1u) == lanes - 1) ? 1u : 0u;
    }
    s_buf[0] = k;
    s_buf[1] = last;
  }
  __syncthreads();
  const uint32_t k = s_buf[0];
  TileClaim r;
  r.ok = (uint64_t)k * kClaimLanes + lane < ntiles;
  r.tile = k * kClaimLanes + lane;
  r.last = s_buf[1] != 0;
  return r;
}

// Thread 0 of the closing block: reset the lane-done counter and publish the epoch.
__device__ __forceinline__ void release_launch(LbState* st, uint32_t epoch) {
  __threadfence();
  __hip_atomic_store(&st->lanes_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&st->epoch, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __threadfence();
}

// ---------------------------------------------------------------------------
// Wave / block scans (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T t = __shfl_up(v, d, kWave);
    if (lane >= d) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive scan over the block; `total` receives the block sum.  `s_wave` needs
// kWavesPerBlock entries.  Contains two barriers.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave, T& total) {
  T incl = wave_incl_scan(v);
  const int wid = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) s_wave[wid] = incl;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) {
    T x = s_wave[i];
    before += (i < wid) ? x : T(0);
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + incl - v;
}

// Wave-parallel lookback: the calling wave (all 64 lanes) sums the values of tiles
// [0, tile) using the status words of up to 64 predecessors per step.  Stops at the
// nearest inclusive prefix.  Sets *err on an expired wait.
__device__ __forceinline__ uint64_t wave_lookback(const uint64_t* status, uint32_t tile,
                                                  uint32_t epoch, uint32_t* err) {
  const int lane = lane_id();
  uint64_t excl = 0;
  int64_t top = (int64_t)tile - 1;
  while (top >= 0) {
    const int64_t idx = top - lane;
    uint64_t val = 0;
    bool incl = true;
    if (idx >= 0) {
      uint32_t spins = 0;
      for (;;) {
        uint64_t s = status_load(status + idx);
        uint64_t flag = s >> 62;
        uint32_t ep = (uint32_t)(s >> 40) & kEpochMask;
        if (flag != 0 && ep == epoch) {
          incl = (flag == 2);
          val = s & kValMask;
          break;
        }
        if (++spins > kSpinLimit) {
          atomicOr(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const uint64_t incl_mask = __ballot(incl);
    if (incl_mask) {
      const int first = __ffsll((unsigned long long)incl_mask) - 1;
      excl = sat_add(excl, wave_sum(lane <= first ? val : 0ull));
      break;
    }
    excl = sat_add(excl, wave_sum(val));
    top -= kWave;
  }
  return excl;
}

// Tile-level exclusive offsets for a single-pass scan: every thread contributes `v`;
// returns the global exclusive prefix of this thread, `grand` gets the inclusive total
// through this tile and `tile_excl` the total of all earlier tiles.  Uses lookback.
struct TileScanShared {
  uint64_t wave[kWavesPerBlock];
  uint64_t excl;
};

__device__ __forceinline__ uint64_t tile_scan(uint64_t v, uint32_t tile, uint32_t epoch,
                                              uint64_t* status, uint32_t* err,
                                              TileScanShared* sh, uint64_t& grand,
                                              uint64_t& tile_excl) {
  uint64_t total;
  uint64_t local = block_excl_scan<uint64_t>(v, sh->wave, total);
  if (threadIdx.x < kWave) {
    if (tile == 0) {
      if (threadIdx.x == 0) {
        status_store(status, status_word(kFlagIncl, epoch, total));
        sh->excl = 0;
      }
    } else {
      if (threadIdx.x == 0) status_store(status + tile, status_word(kFlagAgg, epoch, total));
      uint64_t ex = wave_lookback(status, tile, epoch, err);
      if (threadIdx.x == 0) {
        status_store(status + tile, status_word(kFlagIncl, epoch, sat_add(ex, total)));
        sh->excl = ex;
      }
    }
  }
  __syncthreads();
  uint64_t ex = sh->excl;
  __syncthreads();
  grand = sat_add(ex, total);
  tile_excl = ex;
  return ex + local;
}

// ---------------------------------------------------------------------------
// Binary searches (Section IV-A: at most ceil(log2 n) probes).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ uint64_t lower_bound(const T* a, uint64_t n, T v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ uint64_t upper_bound(const T* a, uint64_t n, T v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Wave-cooperative partition point: all 64 lanes of the calling wave search [lo, hi)
// for the first index whose predicate is false (the predicate holds on a prefix).  Each
// round probes 64 positions at once and narrows the range 65-fold, so a search over
// 5e7 keys takes 5 rounds of parallel loads instead of 26 dependent ones.  The result
// is uniform across the wave.
template <typename Pred>
__device__ __forceinline__ uint64_t wave_partition(uint64_t lo, uint64_t hi, Pred pred) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  while (lo < hi) {
    const uint64_t span = hi - lo;
    if (span <= (uint64_t)kWave) {
      const bool t = (uint64_t)lane < span && pred(lo + (uint64_t)lane);
      return lo + (uint64_t)__popcll(__ballot(t));
    }
    const uint64_t q = lo + (span * (uint64_t)(lane + 1)) / (kWave + 1);
    const uint32_t J = (uint32_t)__popcll(__ballot(pred(q)));
    const uint64_t q_before = lo + (span * (uint64_t)J) / (kWave + 1);
    const uint64_t q_at = lo + (span * (uint64_t)(J + 1)) / (kWave + 1);
    if (J > 0) lo = q_before + 1;
    if (J < (uint32_t)kWave) hi = q_at;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ uint64_t wave_lower_bound(const T* a, uint64_t n, T v) {
  return wave_partition(0, n, [&](uint64_t i) { return a[i] < v; });
}

template <typename T>
__device__ __forceinline__ uint64_t wave_upper_bound(const T* a, uint64_t n, T v) {
  return wave_partition(0, n, [&](uint64_t i) { return a[i] <= v; });
}

// Branchless lower bounds of ITEMS keys at once over the same sorted array: every
// probe step issues ITEMS independent loads, so their latencies overlap.
template <typename T, int ITEMS>
__device__ __forceinline__ void multi_lower_bound(const T* __restrict__ a, uint64_t n,
                                                  const T (&v)[ITEMS], uint64_t (&out)[ITEMS]) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] = 0;
  if (n == 0) return;
  uint64_t len = n;
  while (len > 1) {
    const uint64_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) out[k] = (a[out[k] + half - 1] < v[k]) ? out[k] + half : out[k];
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] += (a[out[k]] < v[k]) ? 1 : 0;
}

template <typename T, int ITEMS>
__device__ __forceinline__ void multi_upper_bound(const T* __restrict__ a, uint64_t n,
                                                  const T (&v)[ITEMS], uint64_t (&out)[ITEMS]) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] = 0;
  if (n == 0) return;
  uint64_t len = n;
  while (len > 1) {
    const uint64_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) out[k] = (a[out[k] + half - 1] <= v[k]) ? out[k] + half : out[k];
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] += (a[out[k]] <= v[k]) ? 1 : 0;
}

// Peers of this lane: lanes of the wave whose 8-bit digit equals this lane's (and that
// are in `active`).  Eight ballots, one per bit.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, uint64_t active) {
  uint64_t peers = active;
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool set = (d >> bit) & 1u;
    const uint64_t m = __ballot(set);
    peers &= set ? m : ~m;
  }
  return peers;
}

// Key field helpers.  `w` < bit width of K always holds (w = 32 only with 64-bit keys).
template <typename K>
__device__ __forceinline__ K field_mask(int w) {
  return (K)((w >= (int)(8 * sizeof(K))) ? ~K(0) : ((K(1) << w) - 1));
}

// Row id of the join vertex of a TC delta key (inst, a, b): (inst << w) | b.
template <typename K>
__device__ __forceinline__ uint32_t tc_join_row(K k, int w) {
  return (uint32_t)((((k >> w) >> w) << w) | (k & field_mask<K>(w)));
}

// Row id of the head of a key: (inst << w) | src.
template <typename K>
__device__ __forceinline__ uint32_t head_row(K k, int w) {
  return (uint32_t)(k >> w);
}

}  // namespace wg
