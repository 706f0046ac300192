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
// Control block and per-iteration records.
//
// Every size that decides a launch lives in device memory.  The host passes each kernel
// of iteration j the number j; the kernel reads what iteration j needs from record j-1
// (written by an earlier launch) and the launch that finishes iteration j writes record
// j.  No field is ever written while other blocks of the same launch may still read it,
// so no launch needs a grid-wide barrier, a blocks-done counter or a lookback chain --
// cross-block handshakes cost microsecond round trips across the XCDs of this chip.
// ---------------------------------------------------------------------------
// Full is kept as two disjoint sorted runs: a large run A and a small run B of recent
// deltas.  Iteration j merges its delta into B -- unless B (non-empty) plus the delta
// would outgrow A / kFoldRatio: then it folds B into A and the delta becomes the new B.
// A is rewritten only when Full has grown by about an eighth, not every iteration as a
// single run would be.
struct IterRec {
  uint64_t N;   // |Delta^j| (record 0: the seed)
  uint64_t C;   // join candidates of iteration j (record 0: base-rule candidates for SG)
  uint64_t F;   // |Full| after iteration j (= |A| + |B|)
  uint64_t FA;  // |A| after iteration j
  uint32_t a;   // buffer side of A after iteration j
  uint32_t b;   // buffer side of B after iteration j
  uint32_t fold;  // iteration j folded B into A (and its delta became B)
  uint32_t tail;  // 1: run by the one-block tail loop; 2: the last of such a launch, whose
                  // new tuples the fold after it merged into B
};

constexpr uint32_t kFoldRatio = 8;  // fold B into A once |B| > |A| / kFoldRatio

struct Ctrl {
  uint64_t m_in;         // input edge count
  uint64_t m_unique;     // |E| after sort + dedup
  uint64_t nu;           // distinct (inst, src) rows of the edge index
  uint64_t cand_cap;     // capacity of each candidate and delta buffer (keys)
  uint64_t full_cap;     // capacity of each Full buffer (keys)
  uint64_t filtered;     // size after the SG diagonal filter
  uint32_t iter;         // highest iteration whose record is complete
  uint32_t max_iter;     // 0: unlimited
  uint32_t done;         // the last delta was empty: fixpoint reached
  uint32_t overflow;     // bit 0 candidates, bit 1 Full, bit 2 delta, bit 3 a one-block
                         // sort enqueued alone found more keys than it holds, bit 4 a
                         // row of the segmented sort is longer than one block holds
  uint32_t limit_hit;    // max_iter reached with a non-empty delta
  uint32_t maxid;        // largest vertex id of the input
  uint32_t force_overflow_at;  // test hook: report a candidate overflow at this iteration
  uint32_t bad_input;          // batched input offsets are malformed
  uint32_t cur;                // iteration in flight (set by its first kernel)
  uint64_t dedup_n;            // unfused variant: candidates left after the dedup pass
  uint64_t cand_n;             // join candidates of the iteration in flight
  uint32_t small_sorted;       // the sort in flight fit one block and is done: the radix
                               // passes of that sort are no-ops
  uint32_t seg_long;           // rows the segmented sort in flight left to its long-row pass
  uint64_t full_n;             // |Full| after the last merged iteration (the seed: |Delta^0|)
  uint64_t tail_n;             // tail loop: size of its run T (0: nothing for the fold)
  uint32_t tail_b;             // ... B's side before the fold (the fold writes the other)
  uint32_t tail_exit;          // ... why it stopped (kTail*)
};

// Why a tail loop stopped: the fixpoint or the iteration limit; the next iteration does
// not fit one block (or the buffers, or is the overflow hook's); run T is full; the
// records the host allotted are used up.
enum : uint32_t { kTailFixpoint = 0, kTailSizes = 1, kTailRun = 2, kTailRecords = 3 };

// Kernels of the loop take their iteration from the device, so that one iteration's
// launches are the same for every iteration (and can be recorded once as a graph): the
// join count, first kernel of an iteration, works on the one after the last completed
// and publishes it; the later kernels read it.  An explicit j (the seed, the base rule,
// the triangle join) is used as given.
constexpr uint32_t kIterDevice = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t iter_begin(Ctrl* c, uint32_t j) {
  if (j != kIterDevice) return j;
  const uint32_t cur = c->iter + 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) c->cur = cur;  // read only by later launches
  return cur;
}

__device__ __forceinline__ uint32_t iter_cur(const Ctrl* c, uint32_t j) {
  return j != kIterDevice ? j : c->cur;
}

// A halted loop turns every later kernel of the batch into a no-op.
__device__ __forceinline__ bool halted(const Ctrl* c) {
  return (c->done | c->overflow | c->limit_hit) != 0;
}

// Early exit of a launch, decided once per block: thread 0's `stop` is the whole block's.
// The flags behind it can be set by another block of the same launch (an overflow, the
// fixpoint, the iteration limit); waves of one block that read them at different moments
// would split, and the waves that stay would meet barriers and block-wide scans whose
// partial sums the others never wrote.  (Blocks may still differ: a block that returns
// because of such a flag has nothing left to contribute once it is set.)
__device__ __forceinline__ bool block_stop(bool stop) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = stop ? 1 : 0;
  __syncthreads();
  return s_stop != 0;
}

// An iteration enqueued with both routes (gate 1: the row route, 2: the sort route; 0: no
// gate): the join's candidate count picks one -- the rows from `row_min` candidates on and
// while Full has at most `full_per_cand` tuples per candidate (the row pass streams each
// touched row of Full; the sort route moves every candidate through the sort passes).
__device__ __forceinline__ bool gated_out(const Ctrl* c, int gate, uint64_t row_min, uint64_t full_per_cand) {
  if (gate == 0) return false;
  const bool row = c->cand_n >= row_min && c->cand_n * full_per_cand >= c->full_n;
  return gate == 1 ? !row : row;
}

constexpr uint64_t kValMask = (1ull << 40) - 1;

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  return s > kValMask ? kValMask : s;
}

// Static tile range of this block: tiles [b*tpb, (b+1)*tpb) of T items each.  Producer
// and consumer launches of one scan use the same n, T and grid, hence the same ranges.
__device__ __forceinline__ void block_range(uint64_t n, uint32_t T, uint64_t& lo, uint64_t& hi) {
  const uint64_t tiles = (n + T - 1) / T;
  const uint64_t tpb = (tiles + gridDim.x - 1) / gridDim.x;
  lo = (uint64_t)blockIdx.x * tpb * T;
  if (lo > n) lo = n;
  hi = lo + tpb * T;
  if (hi > n) hi = n;
}

// Blocks of a G-block launch whose static range is non-empty: exactly blocks
// [0, active_blocks) own keys.
__device__ __forceinline__ uint32_t active_blocks(uint64_t n, uint32_t T, uint32_t G) {
  const uint64_t tiles = (n + T - 1) / T;
  if (tiles == 0) return 0;
  const uint64_t tpb = (tiles + G - 1) / G;
  return (uint32_t)((tiles + tpb - 1) / tpb);
}

// Items per block range for a grid of `G` blocks (what block_range gives every block but
// possibly the last).
__device__ __forceinline__ uint64_t range_len(uint64_t n, uint32_t T, uint32_t G) {
  const uint64_t tiles = (n + T - 1) / T;
  return ((tiles + G - 1) / G) * T;
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
// Largest v of the threads before this one in the block (0 for thread 0).
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t* s_wave) {
  const int lane = lane_id();
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, kWave);
    if (lane >= d) incl = incl > t ? incl : t;
  }
  uint32_t ex = __shfl_up(incl, 1, kWave);
  if (lane == 0) ex = 0;
  const int wid = threadIdx.x / kWave;
  if (lane == kWave - 1) s_wave[wid] = incl;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) {
    const uint32_t x = s_wave[i];
    if (i < wid && x > ex) ex = x;
  }
  __syncthreads();
  return ex;
}

// (WAVES: waves of the block, kWavesPerBlock unless the kernel runs wider blocks;
// s_wave holds WAVES entries)
template <typename T, int WAVES = kWavesPerBlock>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave, T& total) {
  T incl = wave_incl_scan(v);
  const int wid = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) s_wave[wid] = incl;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    T x = s_wave[i];
    before += (i < wid) ? x : T(0);
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + incl - v;
}

// Exclusive prefix sums of the per-block totals vals[0..G) of a producer launch, into
// LDS s_pre[0..G); returns the grand total in every thread.  G <= PER * kBlock.
template <int PER = 4>
__device__ __forceinline__ uint64_t block_prefix(const uint64_t* __restrict__ vals, int G,
                                                 uint64_t* s_pre, uint64_t* s_wave) {
  uint64_t v[PER];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = (int)threadIdx.x * PER + k;
    v[k] = i < G ? vals[i] : 0ull;
    sum = sat_add(sum, v[k]);
  }
  uint64_t total;
  uint64_t ex = block_excl_scan<uint64_t>(sum, s_wave, total);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = (int)threadIdx.x * PER + k;
    if (i < G) s_pre[i] = ex;
    ex = sat_add(ex, v[k]);
  }
  __syncthreads();
  return total;
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
// round splits the range into 64 chunks and probes the last index of each, so a search
// over 5e7 keys takes 5 rounds of parallel loads instead of 26 dependent ones.  Indices
// stay below 2^32 (no relation here holds more keys), so the arithmetic is 32-bit shifts.
// The result is uniform across the wave.
template <typename Pred>
__device__ __forceinline__ uint64_t wave_partition(uint64_t lo64, uint64_t hi64, Pred pred) {
  const uint32_t lane = (uint32_t)(threadIdx.x & (kWave - 1));
  uint32_t lo = (uint32_t)lo64, hi = (uint32_t)hi64;
  while (lo < hi) {
    const uint32_t span = hi - lo;
    if (span <= (uint32_t)kWave) {
      const bool t = lane < span && pred((uint64_t)(lo + lane));
      return lo + (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(t));
    }
    const uint32_t chunk = (span + kWave - 1) >> 6;
    const uint32_t q = lo + (lane + 1) * chunk - 1;  // last index of chunk `lane`
    const bool t = q < hi && pred((uint64_t)q);
    const uint32_t J = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(t));  // chunks wholly before
    const uint32_t qJ = lo + (J + 1) * chunk - 1;  // pred fails here (or qJ >= hi)
    lo += J * chunk;
    if (qJ < hi) hi = qJ;
  }
  return lo;
}

// The same with FAN probes per round until the span fits one 64-lane round: more rounds,
// but each touches FAN scattered lines instead of 64 (for searches whose latency is
// hidden behind other work and whose probed lines would otherwise cost HBM traffic).
template <int FAN, typename Pred>
__device__ __forceinline__ uint64_t wave_partition_fan(uint64_t lo64, uint64_t hi64, Pred pred) {
  static_assert(FAN >= 2 && FAN < kWave, "");
  const uint32_t lane = (uint32_t)(threadIdx.x & (kWave - 1));
  uint32_t lo = (uint32_t)lo64, hi = (uint32_t)hi64;
  while (hi - lo > (uint32_t)kWave) {
    const uint32_t span = hi - lo;
    const uint32_t chunk = (span + FAN - 1) / FAN;
    const uint32_t q = lo + (lane + 1) * chunk - 1;  // last index of chunk `lane`
    const bool t = lane < (uint32_t)FAN && q < hi && pred((uint64_t)q);
    const uint32_t J = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(t));
    const uint32_t qJ = lo + (J + 1) * chunk - 1;
    lo += J * chunk;
    if (qJ < hi) hi = qJ;
  }
  return wave_partition(lo, hi, pred);
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
// probe step issues ITEMS independent loads, so their latencies overlap.  Only the first
// `nk` keys are searched (a count the whole block agrees on; the others get 0).
template <typename T, int ITEMS>
__device__ __forceinline__ void multi_lower_bound(const T* __restrict__ a, uint64_t n,
                                                  const T (&v)[ITEMS], uint64_t (&out)[ITEMS],
                                                  int nk = ITEMS) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] = 0;
  if (n == 0) return;
  uint64_t len = n;
  while (len > 1) {
    const uint64_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (k < nk) out[k] = (a[out[k] + half - 1] < v[k]) ? out[k] + half : out[k];
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (k < nk) out[k] += (a[out[k]] < v[k]) ? 1 : 0;
}

template <typename T, int ITEMS>
__device__ __forceinline__ void multi_upper_bound(const T* __restrict__ a, uint64_t n,
                                                  const T (&v)[ITEMS], uint64_t (&out)[ITEMS],
                                                  int nk = ITEMS) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] = 0;
  if (n == 0) return;
  uint64_t len = n;
  while (len > 1) {
    const uint64_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (k < nk) out[k] = (a[out[k] + half - 1] <= v[k]) ? out[k] + half : out[k];
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (k < nk) out[k] += (a[out[k]] <= v[k]) ? 1 : 0;
}

// multi_upper_bound over a virtual sorted array given by an accessor at(i).
template <int ITEMS, typename At, typename T>
__device__ __forceinline__ void multi_upper_bound_at(At at, uint64_t n, const T (&v)[ITEMS],
                                                     uint64_t (&out)[ITEMS]) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] = 0;
  if (n == 0) return;
  uint64_t len = n;
  while (len > 1) {
    const uint64_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) out[k] = (at(out[k] + half - 1) <= v[k]) ? out[k] + half : out[k];
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] += (at(out[k]) <= v[k]) ? 1 : 0;
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
