// HIP kernels of one semi-naive iteration for gfx950 (CDNA4, wave64).
//
//   join count + scan   Section IV-A, two-phase binary-search join (count phase)
//   join emit           Section IV-A (emit phase) and Section VI (SG cross product)
//   radix pass          Section V-C, LSD radix sort, 8 bits per pass, dst field first
//   dedup_diff          Section IV-B, fused dedup + set difference, ordered compaction
//   merge               Section IV-C, disjoint merge-path merge
//
// Every kernel reads the sizes it works on from the device control block, so a whole
// batch of iterations is enqueued without the host knowing any intermediate size
// (Section V-B).  Kernels that start after the loop halted return at once.
//
// Launch shapes: persistent grids (a few blocks per CU).  Lookback kernels claim tiles
// dynamically over 8 claim lanes; streaming kernels (emit, merge) use a static grid stride.

#include "wg_launch.h"

namespace wg {

constexpr uint32_t kNoRow = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Prepare: largest id, packing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_max_id(Ctrl* ctrl, const uint32_t* __restrict__ src,
                                                   const uint32_t* __restrict__ dst, uint64_t m) {
  uint32_t mx = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * kBlock) {
    mx = max(mx, max(src[i], dst[i]));
  }
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
  if (lane_id() == 0 && mx) atomicMax(&ctrl->maxid, mx);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_pack(const uint32_t* __restrict__ src,
                                                 const uint32_t* __restrict__ dst, uint64_t m,
                                                 int w, K* __restrict__ keys) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * kBlock)
    keys[i] = ((K)src[i] << w) | (K)dst[i];
}

// ---------------------------------------------------------------------------
// Join, count phase (Section IV-A).  One thread per delta tuple finds the range of its
// join key in the edge index by binary search and counts the candidates it will emit;
// a single-pass scan turns the counts into output offsets, so every tuple owns one
// contiguous output slab and the emit phase needs no atomics.  The row ids found here
// are kept for the emit phase instead of searching twice.  Tuples are laid out
// wave-striped (coalesced loads) and all searches of a thread run interleaved.
// ---------------------------------------------------------------------------
template <typename K, int Q, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_join_count(Ctrl* ctrl, Bufs<K> b, int w) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ TileScanShared sh;
  __shared__ uint32_t s_claim[2];
  if (halted(ctrl)) return;
  const uint64_t n = (Q == kJoinSGBase) ? ctrl->nu : ctrl->D;
  const uint64_t nu = ctrl->nu;
  const K* __restrict__ delta = b.delta[ctrl->delta_side];
  const uint32_t* __restrict__ U = b.U;
  const uint32_t* __restrict__ R = b.R;
  const uint64_t ntiles = (n + T - 1) / T;
  if (ntiles == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->C = 0;
    return;
  }
  LbState* st = b.lb + kLbJoin;
  const uint32_t epoch = launch_epoch(st);
  const int wid = threadIdx.x / kWave;
  const int lane = lane_id();
  for (;;) {
    const TileClaim cl = claim_tile(st, ntiles, s_claim);
    if (!cl.ok) {
      if (cl.last && threadIdx.x == 0) release_launch(st, epoch);
      break;
    }
    {
      const uint32_t tile = cl.tile;
      // wave `wid` owns a contiguous run of 64*ITEMS tuples
      const uint64_t wbase = (uint64_t)tile * T + (uint64_t)wid * (kWave * ITEMS);
      uint64_t cnt[ITEMS];
      if (Q == kJoinSGBase) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          const uint64_t i = wbase + (uint64_t)k * kWave + lane;
          uint64_t len = 0;
          if (i < n) len = R[i + 1] - R[i];
          cnt[k] = len ? len * (len - 1) : 0;
        }
      } else {
        uint32_t vb[ITEMS], va[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          const uint64_t i = wbase + (uint64_t)k * kWave + lane;
          const K key = i < n ? delta[i] : K(0);
          vb[k] = tc_join_row<K>(key, w);
          va[k] = head_row<K>(key, w);
        }
        uint64_t jb[ITEMS];
        multi_lower_bound<uint32_t, ITEMS>(U, nu, vb, jb);
        uint64_t ja[ITEMS];
        if (Q == kJoinSG) multi_lower_bound<uint32_t, ITEMS>(U, nu, va, ja);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          const uint64_t i = wbase + (uint64_t)k * kWave + lane;
          uint64_t c = 0;
          if (i < n) {
            const uint32_t rb = (jb[k] < nu && U[jb[k]] == vb[k]) ? (uint32_t)jb[k] : kNoRow;
            b.rowb[i] = rb;
            if (Q == kJoinTC) {
              c = (rb == kNoRow) ? 0 : (uint64_t)(R[rb + 1] - R[rb]);
            } else {
              const uint32_t ra = (ja[k] < nu && U[ja[k]] == va[k]) ? (uint32_t)ja[k] : kNoRow;
              b.rowa[i] = ra;
              c = (ra == kNoRow || rb == kNoRow)
                      ? 0
                      : (uint64_t)(R[ra + 1] - R[ra]) * (uint64_t)(R[rb + 1] - R[rb]);
            }
          }
          cnt[k] = c;
        }
      }
      // exclusive offsets in (k, lane) order inside the wave, then across waves and tiles
      uint64_t ex[ITEMS];
      uint64_t run = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t incl = wave_incl_scan<uint64_t>(cnt[k]);
        ex[k] = run + incl - cnt[k];
        run = sat_add(run, __shfl(incl, kWave - 1, kWave));
      }
      uint64_t grand, tex;
      const uint64_t g = tile_scan(lane == 0 ? run : 0ull, tile, epoch, b.status[kLbJoin],
                                   &ctrl->error, &sh, grand, tex);
      const uint64_t wave_base = __shfl(g, 0, kWave);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t i = wbase + (uint64_t)k * kWave + lane;
        if (i < n) b.off[i] = (uint32_t)sat_add(wave_base, ex[k]);
      }
      if (tile == ntiles - 1 && threadIdx.x == 0) {
        ctrl->C = grand;
        const uint32_t hook = ctrl->force_overflow_at;
        const bool forced = Q != kJoinSGBase && hook != 0 && hook == ctrl->iter + 1;
        if (grand > ctrl->cand_cap || forced) atomicOr(&ctrl->overflow, 1u);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Join, emit phase.  Output positions are dealt out in tiles; each position finds the
// delta tuple that owns it by binary search over the scanned offsets (a load-balanced
// expansion, so a hub tuple with thousands of matches is spread over many threads
// instead of serialising one).  Writes are coalesced.
// ---------------------------------------------------------------------------
template <typename K, int Q, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_join_emit(Ctrl* ctrl, Bufs<K> b, int w) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint32_t s_off[T];
  __shared__ uint64_t s_i0, s_i1;
  if (halted(ctrl)) return;
  const uint64_t C = ctrl->C;
  const uint64_t n = (Q == kJoinSGBase) ? ctrl->nu : ctrl->D;
  const K* __restrict__ delta = b.delta[ctrl->delta_side];
  const uint32_t* __restrict__ off = b.off;
  const uint32_t* __restrict__ R = b.R;
  const uint32_t* __restrict__ Edst = b.Edst;
  K* __restrict__ cand = b.cand[0];
  const uint64_t ntiles = (C + T - 1) / T;
  const int wid = threadIdx.x / kWave;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t p0 = tile * T;
    const uint64_t p1 = min(p0 + T, C);
    // owners of the first and last position of the tile (two waves search concurrently)
    if (wid == 0) {
      const uint64_t i0 = wave_upper_bound(off, n, (uint32_t)p0) - 1;
      if (lane_id() == 0) s_i0 = i0;
    } else if (wid == 1) {
      const uint64_t i1 = wave_upper_bound(off, n, (uint32_t)(p1 - 1)) - 1;
      if (lane_id() == 0) s_i1 = i1;
    }
    __syncthreads();
    const uint64_t i0 = s_i0;
    const uint64_t span = s_i1 - i0 + 1;
    const bool in_lds = span <= T;
    if (in_lds) {
      for (uint32_t j = threadIdx.x; j < span; j += kBlock) s_off[j] = off[i0 + j];
    }
    __syncthreads();
    uint32_t pos[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
      pos[k] = (uint32_t)min(p, p1 - 1);
    }
    uint64_t li[ITEMS];
    if (in_lds) multi_upper_bound<uint32_t, ITEMS>(s_off, span, pos, li);
    else multi_upper_bound<uint32_t, ITEMS>(off + i0, span, pos, li);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
      const bool valid = p < p1;
      K key = 0;
      if (valid) {
        const uint64_t i = i0 + li[k] - 1;
        const uint32_t start = in_lds ? s_off[li[k] - 1] : off[i];
        const uint32_t r = (uint32_t)p - start;
        if (Q == kJoinTC) {
          const K dk = delta[i];
          key = ((dk >> w) << w) | (K)Edst[R[b.rowb[i]] + r];
        } else if (Q == kJoinSG) {
          const K dk = delta[i];
          const uint32_t ja = b.rowa[i], jb = b.rowb[i];
          const uint32_t lb = R[jb + 1] - R[jb];
          const uint32_t qa = r / lb;
          const uint32_t rb = r - qa * lb;
          const K inst = (dk >> w) >> w;
          key = ((((inst << w) | (K)Edst[R[ja] + qa]) << w) | (K)Edst[R[jb] + rb]);
        } else {
          // base rule: ordered pairs (x, y) of distinct children of row i
          const uint32_t len1 = R[i + 1] - R[i] - 1;
          const uint32_t qa = r / len1;
          uint32_t qb = r - qa * len1;
          qb += (qb >= qa) ? 1u : 0u;
          const K inst = (K)(b.U[i] >> w);
          key = ((((inst << w) | (K)Edst[R[i] + qa]) << w) | (K)Edst[R[i] + qb]);
        }
        cand[p] = key;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LSD radix sort (Section V-C): 8 bits per pass, dst field first, every pass stable.
//
// A pass is three launches with no waiting between blocks: count (block b counts the
// digits of a static contiguous range of tiles), scan (one block per digit turns the
// per-block counts into per-block offsets) and scatter (block b re-reads its range tile by
// tile, ranks each tile stably in LDS and writes every key to its final position).
// Chained single-pass scans (decoupled lookback) pay a cross-XCD round trip per
// dependency on this chip; this form pays one extra read of the keys instead, and each
// block writes long per-digit runs of consecutive positions.
// ---------------------------------------------------------------------------

// Static tile range of this block: tiles [b*tpb, (b+1)*tpb) of T keys.
__device__ __forceinline__ void block_range(uint64_t n, uint32_t T, uint64_t& lo, uint64_t& hi) {
  const uint64_t tiles = (n + T - 1) / T;
  const uint64_t tpb = (tiles + gridDim.x - 1) / gridDim.x;
  lo = min(n, (uint64_t)blockIdx.x * tpb * T);
  hi = min(n, lo + tpb * T);
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_count(Ctrl* ctrl, const uint64_t* n_ptr,
                                                        const K* __restrict__ in, int pass,
                                                        uint32_t* __restrict__ cnt) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint32_t s_cnt[kRadix];
  if (halted(ctrl)) return;
  const uint64_t n = *n_ptr;
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const int shift = pass * kRadixBits;
  const uint64_t lt = lanemask_lt();
  for (uint64_t base = lo; base < hi; base += T) {
    K key[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t i = base + (uint64_t)k * kBlock + threadIdx.x;
      key[k] = i < hi ? in[i] : K(0);
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const bool valid = base + (uint64_t)k * kBlock + threadIdx.x < hi;
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
      const uint64_t peers = digit_peers(d, __ballot(valid));
      if (valid && (peers & lt) == 0) atomicAdd(&s_cnt[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  cnt[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = s_cnt[threadIdx.x];
}

// One block per digit: per-block counts of the digit -> exclusive per-block offsets (in
// place); tot[d] = the digit's total.
__global__ __launch_bounds__(kBlock) void k_radix_scan(Ctrl* ctrl, uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ tot, int G) {
  __shared__ uint32_t s_wave[kWavesPerBlock];
  if (halted(ctrl)) return;
  uint32_t* row = cnt + (uint64_t)blockIdx.x * G;
  uint32_t carry = 0;
  for (int base = 0; base < G; base += kBlock) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < G ? row[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<uint32_t>(v, s_wave, total);
    if (i < G) row[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(Ctrl* ctrl, const uint64_t* n_ptr,
                                                          const K* __restrict__ in,
                                                          K* __restrict__ out, int pass,
                                                          const uint32_t* __restrict__ off,
                                                          const uint32_t* __restrict__ tot) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_keys[T];
  __shared__ uint32_t s_cnt[kWavesPerBlock][kRadix];
  __shared__ uint32_t s_loc[kRadix];
  __shared__ uint64_t s_run[kRadix];
  __shared__ uint32_t s_wave[kWavesPerBlock];
  if (halted(ctrl)) return;
  const uint64_t n = *n_ptr;
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  if (lo >= hi) return;
  const int shift = pass * kRadixBits;
  const int tid = threadIdx.x;
  const int wid = tid / kWave;
  const int lane = lane_id();
  const uint64_t lt = lanemask_lt();
  {
    // first position of each digit for this block: digit base + earlier blocks' keys
    const uint32_t t = tot[tid];
    uint32_t all;
    const uint32_t base = block_excl_scan<uint32_t>(t, s_wave, all);
    s_run[tid] = (uint64_t)base + off[(uint64_t)tid * gridDim.x + blockIdx.x];
  }
  for (uint64_t tbase = lo; tbase < hi; tbase += T) {
    for (int j = tid; j < kWavesPerBlock * kRadix; j += kBlock) (&s_cnt[0][0])[j] = 0;
    __syncthreads();
    // wave-striped: wave `wid` owns a contiguous run of 64*ITEMS keys
    const uint64_t wbase = tbase + (uint64_t)wid * (ITEMS * kWave);
    K key[ITEMS];
    uint32_t rank[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t idx = wbase + (uint64_t)k * kWave + lane;
      key[k] = idx < hi ? in[idx] : K(0);
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const bool valid = wbase + (uint64_t)k * kWave + lane < hi;
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
      const uint64_t peers = digit_peers(d, __ballot(valid));
      const uint32_t below = __popcll(peers & lt);
      uint32_t before = 0;
      if (valid) before = s_cnt[wid][d];
      if (valid && below == 0) s_cnt[wid][d] = before + __popcll(peers);
      rank[k] = before + below;
    }
    __syncthreads();
    // thread `tid` owns digit `tid`: per-wave exclusive offsets and the tile total
    uint32_t tile_cnt = 0;
#pragma unroll
    for (int w2 = 0; w2 < kWavesPerBlock; ++w2) {
      const uint32_t c = s_cnt[w2][tid];
      s_cnt[w2][tid] = tile_cnt;
      tile_cnt += c;
    }
    uint32_t total;
    s_loc[tid] = block_excl_scan<uint32_t>(tile_cnt, s_wave, total);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      if (wbase + (uint64_t)k * kWave + lane < hi) {
        const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
        const uint32_t pos = s_loc[d] + s_cnt[wid][d] + rank[k];
        if (pos < T) s_keys[pos] = key[k];
      }
    }
    __syncthreads();
    const uint32_t tile_n = (uint32_t)min<uint64_t>(T, hi - tbase);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t j = (uint32_t)k * kBlock + tid;
      if (j < tile_n) {
        const K kk = s_keys[j];
        const uint32_t d = (uint32_t)(kk >> shift) & (kRadix - 1);
        const uint64_t pos = s_run[d] + (j - s_loc[d]);
        if (pos < n) out[pos] = kk;
      }
    }
    __syncthreads();
    s_run[tid] += tile_cnt;
  }
}

// ---------------------------------------------------------------------------
// Fused dedup + set difference (Section IV-B).  A candidate survives when it is the first
// of its run of equal keys and is absent from Full.  Each tile finds the window of Full
// that can hold its keys with two wave-parallel searches, stages it in LDS when it is
// small, classifies its candidates, and compacts survivors in input order with a
// single-pass scan, so the output stays sorted.
//
// The launch's last claimer publishes the iteration: |Delta^i|, the new Full size and the
// flipped ping-pong sides (Section V-C), so the merge that follows reads its shape from
// the control block and the next iteration starts from the new delta.
// ---------------------------------------------------------------------------
__device__ void dedup_publish(Ctrl* c, int mode, uint64_t cnt, uint64_t* hist) {
  if (mode & kModeIter) {
    const uint64_t F = c->F;
    const uint32_t it = c->iter;
    c->N = cnt;
    if (F + cnt > c->full_cap) { atomicOr(&c->overflow, 2u); return; }
    if (cnt > c->delta_cap) { atomicOr(&c->overflow, 4u); return; }
    if ((uint64_t)it + 2 > c->dsz_cap) { atomicOr(&c->overflow, 8u); return; }
    hist[2 * (uint64_t)(it + 1)] = cnt;
    hist[2 * (uint64_t)(it + 1) + 1] = c->C;
    c->total_cand += c->C;
    c->iter = it + 1;
    if (cnt == 0) {
      c->done = 1;
      return;
    }
    // Delta^i lives in the other delta buffer; Full' goes to the other Full buffer
    c->F = F + cnt;
    c->D = cnt;
    c->full_side ^= 1u;
    c->delta_side ^= 1u;
    if (c->max_iter != 0 && it + 1 >= c->max_iter) c->limit_hit = 1;
    return;
  }
  if (mode & kModeEdges) c->m_unique = cnt;
  if (mode & kModeSeed) {
    c->N = cnt;
    if (cnt > c->full_cap || cnt > c->delta_cap) { atomicOr(&c->overflow, 2u); return; }
    c->F = cnt;
    c->D = cnt;
    c->D0 = cnt;
    c->iter = 0;
    c->total_cand = 0;
    c->full_side = 0;
    c->delta_side = 0;
    hist[0] = cnt;
    hist[1] = (mode & kModeEdges) ? 0 : c->C;
    if (cnt == 0) c->done = 1;
  }
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_dedup_diff(Ctrl* ctrl, int mode, const uint64_t* n_ptr,
                                                       const K* __restrict__ cand, Bufs<K> b) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_c[T + 1];
  __shared__ K s_f[T];
  __shared__ TileScanShared sh;
  __shared__ uint64_t s_flo, s_fhi;
  __shared__ uint32_t s_claim[2];
  if (halted(ctrl)) return;
  const uint64_t n = *n_ptr;
  const bool diff = (mode & kModeIter) != 0;
  const K* __restrict__ full = diff ? b.full[ctrl->full_side] : nullptr;
  const uint64_t F = diff ? ctrl->F : 0;
  K* out1;
  uint64_t cap1;
  K* out2 = nullptr;
  K* out3 = nullptr;
  uint64_t cap2 = 0, cap3 = 0;
  if (diff) {
    out1 = b.delta[ctrl->delta_side ^ 1u];
    cap1 = ctrl->delta_cap;
  } else if (mode & kModeEdges) {
    out1 = b.E;
    cap1 = ctrl->m_in;
    if (mode & kModeSeed) {
      out2 = b.full[0];
      cap2 = ctrl->full_cap;
      out3 = b.delta[0];
      cap3 = ctrl->delta_cap;
    }
  } else {
    out1 = b.full[0];
    cap1 = ctrl->full_cap;
    out2 = b.delta[0];
    cap2 = ctrl->delta_cap;
  }
  const uint64_t ntiles = (n + T - 1) / T;
  if (ntiles == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) dedup_publish(ctrl, mode, 0, b.hist);
    return;
  }
  LbState* st = b.lb + kLbDedup;
  const uint32_t epoch = launch_epoch(st);
  const int wid = threadIdx.x / kWave;
  for (;;) {
    const TileClaim cl = claim_tile(st, ntiles, s_claim);
    if (!cl.ok) {
      if (cl.last && threadIdx.x == 0) {
        __threadfence();
        const uint64_t total = __hip_atomic_load(&ctrl->total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        dedup_publish(ctrl, mode, total, b.hist);
        release_launch(st, epoch);
      }
      break;
    }
    {
      const uint32_t tile = cl.tile;
      const uint64_t tbase = (uint64_t)tile * T;
      const uint32_t tn = (uint32_t)min<uint64_t>(T, n - tbase);
      for (uint32_t j = threadIdx.x; j < tn; j += kBlock) s_c[j + 1] = cand[tbase + j];
      if (threadIdx.x == 0 && tile > 0) s_c[0] = cand[tbase - 1];
      if (diff) {
        // window of Full that can hold this tile's keys (two waves search concurrently)
        if (wid == 0) {
          const uint64_t flo = wave_lower_bound(full, F, cand[tbase]);
          if (lane_id() == 0) s_flo = flo;
        } else if (wid == 1) {
          const uint64_t fhi = wave_upper_bound(full, F, cand[tbase + tn - 1]);
          if (lane_id() == 0) s_fhi = fhi;
        }
      }
      __syncthreads();
      uint64_t flo = 0, fspan = 0;
      bool win = false;
      if (diff) {
        flo = s_flo;
        fspan = s_fhi > flo ? s_fhi - flo : 0;
        win = fspan <= T;
        if (win) {
          for (uint32_t j = threadIdx.x; j < fspan; j += kBlock) s_f[j] = full[flo + j];
        }
        __syncthreads();
      }
      uint32_t keep_mask = 0, cnt = 0;
      const uint32_t j0 = threadIdx.x * ITEMS;
      K cv[ITEMS];
      bool dup[ITEMS];
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t j = j0 + k;
        cv[k] = (j < tn) ? s_c[j + 1] : K(0);
        dup[k] = (j >= tn) || !((tbase + j == 0) || (cv[k] != s_c[j]));
      }
      bool member[ITEMS];
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) member[k] = false;
      if (fspan > 0) {
        uint64_t pos[ITEMS];
        if (win) {
          multi_lower_bound<K, ITEMS>(s_f, fspan, cv, pos);
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) member[k] = pos[k] < fspan && s_f[pos[k]] == cv[k];
        } else {
          multi_lower_bound<K, ITEMS>(full + flo, fspan, cv, pos);
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) member[k] = pos[k] < fspan && full[flo + pos[k]] == cv[k];
        }
      }
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (!dup[k] && !member[k]) {
          keep_mask |= 1u << k;
          ++cnt;
        }
      }
      uint64_t grand, tex;
      const uint64_t g = tile_scan(cnt, tile, epoch, b.status[kLbDedup], &ctrl->error, &sh, grand, tex);
      // tile_scan ends with a barrier, so s_f is free to reuse for the survivors.
      uint32_t lpos = (uint32_t)(g - tex);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if ((keep_mask >> k) & 1u) s_f[lpos++] = cv[k];
      __syncthreads();
      const uint32_t tcount = (uint32_t)(grand - tex);
      for (uint32_t j = threadIdx.x; j < tcount; j += kBlock) {
        const uint64_t p = tex + j;
        const K v = s_f[j];
        if (p < cap1) out1[p] = v;
        if (out2 && p < cap2) out2[p] = v;
        if (out3 && p < cap3) out3[p] = v;
      }
      if (tile == ntiles - 1 && threadIdx.x == 0)
        __hip_atomic_store(&ctrl->total, grand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Disjoint merge (Section IV-C).  Full and the new delta are disjoint by construction, so
// Full' has exactly |Full| + |Delta| keys and each tile's slice of both inputs is fixed by
// a merge-path diagonal search: no atomics, no cleanup pass.  Tiles that take keys from
// one input only are straight copies.  The sizes and sides were published by dedup_diff:
// Full' goes to full[full_side], the old Full is the other buffer.
// ---------------------------------------------------------------------------
// Number of A keys among the first `diag` keys of merge(A, B), found by the whole wave.
template <typename K>
__device__ __forceinline__ uint64_t wave_merge_path(const K* A, uint64_t na, const K* B, uint64_t nb,
                                                    uint64_t diag) {
  const uint64_t lo = diag > nb ? diag - nb : 0;
  const uint64_t hi = diag < na ? diag : na;
  return wave_partition(lo, hi, [&](uint64_t i) { return A[i] < B[diag - 1 - i]; });
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_merge(Ctrl* ctrl, Bufs<K> b) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_in[T];
  __shared__ K s_out[T];
  __shared__ uint64_t s_i0, s_i1;
  if (halted(ctrl)) return;
  const uint64_t total = ctrl->F;
  const uint64_t nb = ctrl->N;
  const uint64_t na = total - nb;
  const uint32_t fs = ctrl->full_side, ds = ctrl->delta_side;
  const K* __restrict__ A = b.full[fs ^ 1u];
  const K* __restrict__ B = b.delta[ds];
  K* __restrict__ O = b.full[fs];
  const uint64_t ntiles = (total + T - 1) / T;
  const int wid = threadIdx.x / kWave;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t o0 = tile * T;
    const uint64_t o1 = min(o0 + T, total);
    if (wid == 0) {
      const uint64_t i0 = wave_merge_path(A, na, B, nb, o0);
      if (lane_id() == 0) s_i0 = i0;
    } else if (wid == 1) {
      const uint64_t i1 = wave_merge_path(A, na, B, nb, o1);
      if (lane_id() == 0) s_i1 = i1;
    }
    __syncthreads();
    const uint64_t i0 = s_i0, i1 = s_i1;
    const uint64_t j0 = o0 - i0, j1 = o1 - i1;
    const uint32_t ca = (uint32_t)(i1 - i0), cb = (uint32_t)(j1 - j0);
    if (cb == 0) {
      for (uint32_t t = threadIdx.x; t < ca; t += kBlock) O[o0 + t] = A[i0 + t];
    } else if (ca == 0) {
      for (uint32_t t = threadIdx.x; t < cb; t += kBlock) O[o0 + t] = B[j0 + t];
    } else {
      const uint32_t cn = ca + cb;
      for (uint32_t t = threadIdx.x; t < cn; t += kBlock)
        s_in[t] = t < ca ? A[i0 + t] : B[j0 + (t - ca)];
      __syncthreads();
      const uint32_t dg = threadIdx.x * ITEMS;
      if (dg < cn) {
        uint32_t lo = dg > cb ? dg - cb : 0;
        uint32_t hi = dg < ca ? dg : ca;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_in[mid] < s_in[ca + dg - 1 - mid]) lo = mid + 1; else hi = mid;
        }
        uint32_t ia = lo, ib = dg - lo;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          if (dg + k < cn) {
            const bool take_a = ib >= cb || (ia < ca && s_in[ia] < s_in[ca + ib]);
            s_out[dg + k] = take_a ? s_in[ia++] : s_in[ca + ib++];
          }
        }
      }
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < cn; t += kBlock) O[o0 + t] = s_out[t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Edge index: E is sorted once and never modified (Section IV-A), so the edges of each
// (inst, src) row are contiguous.  U lists the distinct rows, R their starts.
// ---------------------------------------------------------------------------
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_edge_index(Ctrl* ctrl, Bufs<K> b, int w) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ TileScanShared sh;
  __shared__ uint32_t s_claim[2];
  if (ctrl->error | ctrl->overflow) return;
  const uint64_t n = ctrl->m_unique;
  const K* __restrict__ E = b.E;
  const K mask = field_mask<K>(w);
  const uint64_t ntiles = (n + T - 1) / T;
  if (ntiles == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->nu = 0;
      b.R[0] = 0;
    }
    return;
  }
  LbState* st = b.lb + kLbIndex;
  const uint32_t epoch = launch_epoch(st);
  for (;;) {
    const TileClaim cl = claim_tile(st, ntiles, s_claim);
    if (!cl.ok) {
      if (cl.last && threadIdx.x == 0) release_launch(st, epoch);
      break;
    }
    {
      const uint32_t tile = cl.tile;
      const uint64_t base = (uint64_t)tile * T + (uint64_t)threadIdx.x * ITEMS;
      uint32_t heads = 0, cnt = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t i = base + k;
        if (i < n) {
          const K e = E[i];
          b.Edst[i] = (uint32_t)(e & mask);
          if (i == 0 || (e >> w) != (E[i - 1] >> w)) {
            heads |= 1u << k;
            ++cnt;
          }
        }
      }
      uint64_t grand, tex;
      uint64_t g = tile_scan(cnt, tile, epoch, b.status[kLbIndex], &ctrl->error, &sh, grand, tex);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if ((heads >> k) & 1u) {
          const uint64_t i = base + k;
          b.U[g] = (uint32_t)(E[i] >> w);
          b.R[g] = (uint32_t)i;
          ++g;
        }
      }
      if (tile == ntiles - 1 && threadIdx.x == 0) {
        ctrl->nu = grand;
        b.R[grand] = (uint32_t)n;
      }
    }
  }
}

// SG with WG_SG_IRREFLEXIVE: drop (x, x) from the final relation (Full -> other side).
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_filter_offdiag(Ctrl* ctrl, Bufs<K> b, int w) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ TileScanShared sh;
  __shared__ K s_out[T];
  __shared__ uint32_t s_claim[2];
  if (ctrl->error) return;
  const uint64_t n = ctrl->F;
  const uint32_t fs = ctrl->full_side;
  const K* __restrict__ in = b.full[fs];
  K* __restrict__ out = b.full[fs ^ 1u];
  const K mask = field_mask<K>(w);
  const uint64_t ntiles = (n + T - 1) / T;
  if (ntiles == 0) return;
  LbState* st = b.lb + kLbFilter;
  const uint32_t epoch = launch_epoch(st);
  for (;;) {
    const TileClaim cl = claim_tile(st, ntiles, s_claim);
    if (!cl.ok) {
      if (cl.last && threadIdx.x == 0) {
        __threadfence();
        ctrl->F = __hip_atomic_load(&ctrl->total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ctrl->full_side = fs ^ 1u;
        release_launch(st, epoch);
      }
      break;
    }
    {
      const uint32_t tile = cl.tile;
      const uint64_t base = (uint64_t)tile * T + (uint64_t)threadIdx.x * ITEMS;
      uint32_t keep = 0, cnt = 0;
      K v[ITEMS];
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t i = base + k;
        v[k] = 0;
        if (i < n) {
          v[k] = in[i];
          if (((v[k] >> w) & mask) != (v[k] & mask)) {
            keep |= 1u << k;
            ++cnt;
          }
        }
      }
      uint64_t grand, tex;
      const uint64_t g = tile_scan(cnt, tile, epoch, b.status[kLbFilter], &ctrl->error, &sh, grand, tex);
      uint32_t lpos = (uint32_t)(g - tex);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if ((keep >> k) & 1u) s_out[lpos++] = v[k];
      __syncthreads();
      const uint32_t tcount = (uint32_t)(grand - tex);
      for (uint32_t j = threadIdx.x; j < tcount; j += kBlock) out[tex + j] = s_out[j];
      if (tile == ntiles - 1 && threadIdx.x == 0)
        __hip_atomic_store(&ctrl->total, grand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
    }
  }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_unpack(const K* __restrict__ keys, uint64_t n, int w,
                                                   uint32_t* __restrict__ src,
                                                   uint32_t* __restrict__ dst) {
  const K mask = field_mask<K>(w);
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    const K k = keys[i];
    src[i] = (uint32_t)((k >> w) & mask);
    dst[i] = (uint32_t)(k & mask);
  }
}

__global__ void k_resume(Ctrl* ctrl, uint64_t cand_cap, uint64_t full_cap, uint64_t dsz_cap,
                         uint32_t clear_hook) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctrl->cand_cap = cand_cap;
    ctrl->delta_cap = cand_cap;
    ctrl->full_cap = full_cap;
    ctrl->dsz_cap = dsz_cap;
    ctrl->overflow = 0;
    if (clear_hook) ctrl->force_overflow_at = 0;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline int stream_blocks(const Grid& g, uint64_t n) {
  const uint64_t need = (n + kBlock - 1) / kBlock;
  return (int)(need < (uint64_t)g.stream ? (need ? need : 1) : (uint64_t)g.stream);
}

void launch_max_id(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint32_t* src,
                   const uint32_t* dst, uint64_t m) {
  hipLaunchKernelGGL(k_max_id, dim3(stream_blocks(g, m)), dim3(kBlock), 0, s, ctrl, src, dst, m);
}

template <typename K>
void launch_pack(hipStream_t s, const Grid& g, const uint32_t* src, const uint32_t* dst,
                 uint64_t m, int w, K* keys) {
  hipLaunchKernelGGL(k_pack<K>, dim3(stream_blocks(g, m)), dim3(kBlock), 0, s, src, dst, m, w, keys);
}

template <typename K>
void launch_join_count(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w) {
  if (kind == kJoinTC)
    hipLaunchKernelGGL((k_join_count<K, kJoinTC, kJoinItems>), dim3(g.persistent), dim3(kBlock), 0, s, ctrl, b, w);
  else if (kind == kJoinSG)
    hipLaunchKernelGGL((k_join_count<K, kJoinSG, kJoinItems>), dim3(g.persistent), dim3(kBlock), 0, s, ctrl, b, w);
  else
    hipLaunchKernelGGL((k_join_count<K, kJoinSGBase, kJoinItems>), dim3(g.persistent), dim3(kBlock), 0, s, ctrl, b, w);
}

template <typename K>
void launch_join_emit(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w) {
  if (kind == kJoinTC)
    hipLaunchKernelGGL((k_join_emit<K, kJoinTC, kEmitItems>), dim3(g.stream), dim3(kBlock), 0, s, ctrl, b, w);
  else if (kind == kJoinSG)
    hipLaunchKernelGGL((k_join_emit<K, kJoinSG, kEmitItems>), dim3(g.stream), dim3(kBlock), 0, s, ctrl, b, w);
  else
    hipLaunchKernelGGL((k_join_emit<K, kJoinSGBase, kEmitItems>), dim3(g.stream), dim3(kBlock), 0, s, ctrl, b, w);
}

template <typename K>
void launch_radix_pass(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr,
                       const K* in, K* out, int pass, const Bufs<K>& b) {
  constexpr int ITEMS = pass_items<K>();
  hipLaunchKernelGGL((k_radix_count<K, ITEMS>), dim3(g.sort), dim3(kBlock), 0, s, ctrl, n_ptr, in,
                     pass, b.rcnt);
  hipLaunchKernelGGL(k_radix_scan, dim3(kRadix), dim3(kBlock), 0, s, ctrl, b.rcnt, b.rtot, g.sort);
  hipLaunchKernelGGL((k_radix_scatter<K, ITEMS>), dim3(g.sort), dim3(kBlock), 0, s, ctrl, n_ptr, in,
                     out, pass, b.rcnt, b.rtot);
}

template <typename K>
void launch_dedup_diff(hipStream_t s, const Grid& g, int mode, Ctrl* ctrl, const uint64_t* n_ptr,
                       const K* cand, const Bufs<K>& b) {
  hipLaunchKernelGGL((k_dedup_diff<K, kDedupItems>), dim3(g.persistent), dim3(kBlock), 0, s, ctrl,
                     mode, n_ptr, cand, b);
}

template <typename K>
void launch_merge(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b) {
  hipLaunchKernelGGL((k_merge<K, kMergeItems>), dim3(g.stream), dim3(kBlock), 0, s, ctrl, b);
}

template <typename K>
void launch_edge_index(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w) {
  hipLaunchKernelGGL((k_edge_index<K, kIndexItems>), dim3(g.persistent), dim3(kBlock), 0, s, ctrl, b, w);
}

template <typename K>
void launch_filter_offdiag(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w) {
  hipLaunchKernelGGL((k_filter_offdiag<K, kIndexItems>), dim3(g.persistent), dim3(kBlock), 0, s, ctrl, b, w);
}

template <typename K>
void launch_unpack(hipStream_t s, const Grid& g, const K* keys, uint64_t n, int w, uint32_t* src,
                   uint32_t* dst) {
  hipLaunchKernelGGL(k_unpack<K>, dim3(stream_blocks(g, n)), dim3(kBlock), 0, s, keys, n, w, src, dst);
}

void launch_resume(hipStream_t s, Ctrl* ctrl, uint64_t cand_cap, uint64_t full_cap,
                   uint64_t dsz_cap, uint32_t clear_hook) {
  hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, ctrl, cand_cap, full_cap, dsz_cap, clear_hook);
}

#define WG_INSTANTIATE(K)                                                                          \
  template void launch_pack<K>(hipStream_t, const Grid&, const uint32_t*, const uint32_t*,       \
                               uint64_t, int, K*);                                                \
  template void launch_join_count<K>(hipStream_t, const Grid&, int, Ctrl*, const Bufs<K>&, int);   \
  template void launch_join_emit<K>(hipStream_t, const Grid&, int, Ctrl*, const Bufs<K>&, int);    \
  template void launch_radix_pass<K>(hipStream_t, const Grid&, Ctrl*, const uint64_t*, const K*,   \
                                     K*, int, const Bufs<K>&);                                     \
  template void launch_dedup_diff<K>(hipStream_t, const Grid&, int, Ctrl*, const uint64_t*,        \
                                     const K*, const Bufs<K>&);                                    \
  template void launch_merge<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&);                  \
  template void launch_edge_index<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&, int);        \
  template void launch_filter_offdiag<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&, int);    \
  template void launch_unpack<K>(hipStream_t, const Grid&, const K*, uint64_t, int, uint32_t*,     \
                                 uint32_t*);

WG_INSTANTIATE(uint32_t)
WG_INSTANTIATE(uint64_t)

}  // namespace wg
