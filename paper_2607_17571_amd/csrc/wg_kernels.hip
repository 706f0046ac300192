// HIP kernels of one semi-naive iteration for gfx950 (CDNA4, wave64).
//
//   join count, emit    Section IV-A, two-phase binary-search join; Section VI (SG)
//   radix count/scan/   Section V-C, LSD radix sort, 8 bits per pass, dst field first
//     scatter
//   compact local/      Section IV-B, fused dedup + set difference, ordered compaction
//     gather
//   merge               Section IV-C, disjoint merge-path merge
//
// Every kernel reads the sizes it works on from device memory (the control block and
// the per-iteration records), so whole batches of iterations are enqueued without the
// host knowing any intermediate size (Section V-B).  Kernels that start after the loop
// halted return at once.
//
// Scans across blocks are two launches, never a chain inside one launch: a producer in
// which block b handles a static contiguous range and writes its total, and a consumer
// in which every block adds up the totals of the blocks before it.  On this chip a
// cross-block handshake (same-address atomics, lookback polling across the XCDs' L2s)
// costs a microsecond-scale round trip, which a chained scan pays once per tile.

#include <hip/hip_ext.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "../../include/wg.h"
#include "wg_internal.h"
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

// Batched input: instance i owns edges [offsets[i], offsets[i+1]).  Malformed offsets
// (not starting at 0, decreasing, or not ending at m) set ctrl->bad_input.
__global__ __launch_bounds__(kBlock) void k_check_offsets(Ctrl* ctrl, const uint64_t* __restrict__ offsets,
                                                          uint32_t num, uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < num;
       i += (uint64_t)gridDim.x * kBlock) {
    const bool bad = offsets[i] > offsets[i + 1] || (i == 0 && offsets[0] != 0) ||
                     (i + 1 == num && offsets[num] != m);
    if (bad) ctrl->bad_input = 1;
  }
}

// key = inst << 2w | src << w | dst, with inst the instance owning edge i: the number of
// instance ends offsets[1..num] at or below i.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_pack_batch(const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ dst, uint64_t m,
                                                       int w, const uint64_t* __restrict__ offsets,
                                                       uint32_t num, K* __restrict__ keys) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * kBlock) {
    const K inst = (K)upper_bound<uint64_t>(offsets + 1, num, i);
    keys[i] = (((inst << w) | (K)src[i]) << w) | (K)dst[i];
  }
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
// Join, count phase (Section IV-A).  Each delta tuple finds the range of its join key in
// the edge index and counts the candidates it will emit: by binary search over the
// distinct rows U, or, when the row ids span a small enough range, by two loads from a
// dense index whose entry v is the first edge of row v.  Block b owns
// a static range of tuples and writes, per tuple, the offset of its slab relative to the
// range and, per block, the range's total; the emit phase adds the totals of earlier
// blocks, so every tuple owns one contiguous output slab and no atomics are needed.  The
// row ids found here are kept for the emit phase instead of searching twice.  Tuples are
// laid out wave-striped (coalesced loads) and a thread's searches run interleaved.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool row_found(const uint32_t* __restrict__ U, uint64_t nu, uint64_t j,
                                          uint32_t v) {
  return j < nu && U[j] == v;
}

// ---------------------------------------------------------------------------
// Fair hash variant of the join (WG_JOIN_HASH_ROWS): the sorted join's structure with its row
// lookups through hash tables instead of the index.  The row table maps each distinct row
// of E to its index among the rows (its edges are contiguous in E: R[index] .. R[index+1]),
// so a lookup is one expected probe, and the emit stays load-balanced over the outputs; the
// pair set holds every key of E, for triangle counting's closing-edge test.  Open
// addressing, linear probing, load at most 1/2; a slot holds (row << 32 | index), or a key,
// and kHashVacant never equals either (indices stay below 2^32 - 16, keys below 2^63).
// ---------------------------------------------------------------------------
constexpr uint64_t kHashVacant = ~0ull;

__device__ __forceinline__ uint32_t mix_slot(uint64_t x, uint32_t mask) {
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  x ^= x >> 33;
  x *= 0xC4CEB9FE1A85EC53ull;
  x ^= x >> 33;
  return (uint32_t)x & mask;
}

// Index of `row` among E's distinct rows, or kNoRow.
__device__ __forceinline__ uint32_t hash_row_find(const uint64_t* __restrict__ t, uint32_t mask, uint32_t row) {
  for (uint32_t slot = mix_slot(row, mask);; slot = (slot + 1) & mask) {
    const uint64_t e = t[slot];
    if (e == kHashVacant) return 0xFFFFFFFFu;
    if ((uint32_t)(e >> 32) == row) return (uint32_t)e;
  }
}

// Whether `key` is in the pair set.
__device__ __forceinline__ bool hash_pair_has(const uint64_t* __restrict__ t, uint32_t mask, uint64_t key) {
  for (uint32_t slot = mix_slot(key, mask);; slot = (slot + 1) & mask) {
    const uint64_t e = t[slot];
    if (e == kHashVacant) return false;
    if (e == key) return true;
  }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_hash_rows_build(Ctrl* ctrl, Bufs<K> b) {
  if (block_stop(halted(ctrl))) return;
  const uint64_t nu = ctrl->nu;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nu; i += (uint64_t)gridDim.x * kBlock) {
    const uint32_t row = b.U[i];
    const uint64_t entry = ((uint64_t)row << 32) | i;
    uint32_t slot = mix_slot(row, b.hrows);
    while (atomicCAS((unsigned long long*)&b.htab[slot], (unsigned long long)kHashVacant,
                     (unsigned long long)entry) != (unsigned long long)kHashVacant)
      slot = (slot + 1) & b.hrows;
  }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_hash_pairs_build(Ctrl* ctrl, Bufs<K> b) {
  if (block_stop(halted(ctrl))) return;
  const uint64_t mu = ctrl->m_unique;
  uint64_t* __restrict__ t = b.htab + (uint64_t)b.hrows + 1;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < mu; i += (uint64_t)gridDim.x * kBlock) {
    const uint64_t key = (uint64_t)b.E[i];
    uint32_t slot = mix_slot(key, b.hpairs);
    while (atomicCAS((unsigned long long*)&t[slot], (unsigned long long)kHashVacant, (unsigned long long)key) !=
           (unsigned long long)kHashVacant)
      slot = (slot + 1) & b.hpairs;
  }
}

template <typename K, int Q, int ITEMS, bool HR = false>
__global__ __launch_bounds__(kBlock) void k_join_count(Ctrl* ctrl, Bufs<K> b, int w, uint32_t j) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint64_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl))) return;
  j = iter_begin(ctrl, j);
  const uint64_t n = (Q == kJoinSGBase) ? ctrl->nu : b.rec[j - 1].N;
  const uint64_t nu = ctrl->nu;
  const bool dense = b.dense != 0;
  const K* __restrict__ delta = b.delta[(j - 1) & 1u];
  const uint32_t* __restrict__ U = b.U;
  const uint32_t* __restrict__ R = b.R;
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  const int wid = threadIdx.x / kWave;
  const int lane = lane_id();
  uint64_t running = 0;
  for (uint64_t tbase = lo; tbase < hi; tbase += T) {
    const uint64_t wbase = tbase + (uint64_t)wid * (kWave * ITEMS);
    uint64_t cnt[ITEMS];
    if (Q == kJoinSGBase) {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t i = wbase + (uint64_t)k * kWave + lane;
        uint64_t len = 0;
        if (i < hi) len = R[i + 1] - R[i];
        cnt[k] = len ? len * (len - 1) : 0;
      }
    } else {
      uint32_t vb[ITEMS], va[ITEMS];
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t i = wbase + (uint64_t)k * kWave + lane;
        const K key = i < hi ? delta[i] : K(0);
        vb[k] = tc_join_row<K>(key, w);
        va[k] = head_row<K>(key, w);
      }
      uint64_t jb[ITEMS], ja[ITEMS];
      if (!dense) {
        if constexpr (HR) {
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) jb[k] = hash_row_find(b.htab, b.hrows, vb[k]);
        } else {
          multi_lower_bound<uint32_t, ITEMS>(U, nu, vb, jb);
          if (Q == kJoinSG) multi_lower_bound<uint32_t, ITEMS>(U, nu, va, ja);
        }
      }
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t i = wbase + (uint64_t)k * kWave + lane;
        uint64_t c = 0;
        if (i < hi) {
          // dense index: the row id is the vertex id itself (every id below b.dense)
          const uint32_t rb = dense ? vb[k]
                                    : (HR ? (uint32_t)jb[k]
                                          : (row_found(U, nu, jb[k], vb[k]) ? (uint32_t)jb[k] : kNoRow));
          if (!dense) b.rowb[i] = rb;
          if (Q == kJoinTC) {
            c = (rb == kNoRow) ? 0 : (uint64_t)(R[rb + 1] - R[rb]);
          } else {
            const uint32_t ra =
                dense ? va[k] : (row_found(U, nu, ja[k], va[k]) ? (uint32_t)ja[k] : kNoRow);
            if (!dense) b.rowa[i] = ra;
            c = (ra == kNoRow || rb == kNoRow)
                    ? 0
                    : (uint64_t)(R[ra + 1] - R[ra]) * (uint64_t)(R[rb + 1] - R[rb]);
          }
        }
        cnt[k] = c;
      }
    }
    // exclusive offsets in (k, lane) order inside the wave, then across the waves
    uint64_t ex[ITEMS];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t incl = wave_incl_scan<uint64_t>(cnt[k]);
      ex[k] = run + incl - cnt[k];
      run = sat_add(run, __shfl(incl, kWave - 1, kWave));
    }
    uint64_t tile_total;
    const uint64_t g = block_excl_scan<uint64_t>(lane == 0 ? run : 0ull, s_wave, tile_total);
    const uint64_t wave_base = sat_add(running, __shfl(g, 0, kWave));
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t i = wbase + (uint64_t)k * kWave + lane;
      if (i < hi) b.off[i] = (uint32_t)sat_add(wave_base, ex[k]);
    }
    running = sat_add(running, tile_total);
  }
  if (threadIdx.x == 0) b.jtot[blockIdx.x] = running;
}

// ---------------------------------------------------------------------------
// Join, emit phase.  Every block first adds up the per-block totals of the count phase
// (the candidate total C, and the slab base of every count block).  Output positions are
// dealt out in tiles of T; the tuples whose slabs meet a tile are found by two searches
// over the slab offsets, and, when there are at most T of them, each is looked up once
// into LDS (slab start, key bits it passes on, first edge of its join row).  Every
// position then finds its tuple by a max-scan over the slab starts marked in the tile (a
// load-balanced expansion: a hub tuple with thousands of matches is spread over many
// threads instead of serialising one), and reads one edge.  Writes are coalesced.
// ---------------------------------------------------------------------------
template <typename K, int Q, int ITEMS, bool HR = false>
__global__ __launch_bounds__(kBlock) void k_join_emit(Ctrl* ctrl, Bufs<K> b, int w, uint32_t j,
                                                      int gc) {
  constexpr uint32_t T = kBlock * ITEMS;
  constexpr bool kSG = Q == kJoinSG || Q == kJoinSGBase;
  static_assert(T <= 65536, "tuple indices within a tile are kept in 16 bits");
  __shared__ uint64_t s_pre[kScanBlocksMax];
  __shared__ uint64_t s_wave[kWavesPerBlock];
  __shared__ uint16_t s_own[T];             // per position of the tile: its tuple (from i0, < T)
  __shared__ uint32_t s_start[T];           // per staged tuple: first position
  __shared__ uint32_t s_base[T];            // per staged tuple: first edge of the join row
  __shared__ uint32_t s_aux[kSG ? T : 1];   // SG: first edge of the head row
  __shared__ uint32_t s_len[kSG ? T : 1];   // SG: divisor of the pair index
  __shared__ K s_head[T];                   // per staged tuple: key bits passed on
  __shared__ uint64_t s_i0, s_i1;
  if (block_stop(halted(ctrl))) return;
  j = iter_cur(ctrl, j);
  const uint64_t n = (Q == kJoinSGBase) ? ctrl->nu : b.rec[j - 1].N;
  const uint64_t C = block_prefix(b.jtot, gc, s_pre, s_wave);
  const uint32_t hook = ctrl->force_overflow_at;
  const bool forced = Q != kJoinSGBase && Q != kJoinTri && hook != 0 && hook == j;
  // candidates are stored (all but the probe), and positions are 32-bit
  const bool over = Q == kJoinTri ? C > 0xFFFFFFFFull : C > ctrl->cand_cap;
  if (over || forced) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      b.rec[j].C = C;
      atomicOr(&ctrl->overflow, 1u);
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    b.rec[j].C = C;
    ctrl->cand_n = C;
  }
  const bool dense = b.dense != 0;
  const K* __restrict__ delta = b.delta[(j - 1) & 1u];
  const uint32_t* __restrict__ off = b.off;
  const uint32_t* __restrict__ R = b.R;
  const uint32_t* __restrict__ Edst = b.Edst;
  const K mask = field_mask<K>(w);
  K* __restrict__ cand = b.cand[0];
  const uint64_t Pc = range_len(n, kJoinTile, (uint32_t)gc);
  // first candidate of tuple i
  auto at = [&](uint64_t i) -> uint64_t { return s_pre[i / Pc] + off[i]; };
  // join rows of tuple i: rb (the row its candidates come from), ra (SG: the head row)
  auto row_b = [&](uint64_t i, K dk) -> uint32_t { return dense ? tc_join_row<K>(dk, w) : b.rowb[i]; };
  auto row_a = [&](uint64_t i, K dk) -> uint32_t { return dense ? head_row<K>(dk, w) : b.rowa[i]; };
  // whether the closing edge (c, a) of a two-path is in E (kJoinTri)
  auto closes = [&](K dk, K c) -> bool {
    const K a = (dk >> w) & mask;
    const K inst = (dk >> w) >> w;
    if constexpr (HR) {
      return hash_pair_has(b.htab + (uint64_t)b.hrows + 1, b.hpairs, (uint64_t)((((inst << w) | c) << w) | a));
    }
    if (dense) {
      const uint32_t rc = (uint32_t)((inst << w) | c);
      uint32_t lo = R[rc];
      uint32_t len = R[rc + 1] - lo;
      while (len > 0) {
        const uint32_t half = len >> 1;
        if ((K)Edst[lo + half] < a) {
          lo += half + 1;
          len -= half + 1;
        } else {
          len = half;
        }
      }
      return len == 0 && lo < R[rc + 1] && (K)Edst[lo] == a;
    }
    const K probe = (((inst << w) | c) << w) | a;
    const uint64_t mu = ctrl->m_unique;
    uint64_t lo = 0, len = mu;
    while (len > 0) {
      const uint64_t half = len >> 1;
      if (b.E[lo + half] < probe) {
        lo += half + 1;
        len -= half + 1;
      } else {
        len = half;
      }
    }
    return lo < mu && b.E[lo] == probe;
  };
  const uint64_t ntiles = (C + T - 1) / T;
  const int wid = threadIdx.x / kWave;
  uint64_t hits = 0;  // kJoinTri: closing edges found by this thread
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t p0 = tile * T;
    const uint64_t p1 = min(p0 + T, C);
    // owners of the first and last position of the tile (two waves search concurrently)
    if (wid == 0) {
      const uint64_t i0 = wave_partition(0, n, [&](uint64_t i) { return at(i) <= p0; }) - 1;
      if (lane_id() == 0) s_i0 = i0;
    } else if (wid == 1) {
      const uint64_t i1 = wave_partition(0, n, [&](uint64_t i) { return at(i) <= p1 - 1; }) - 1;
      if (lane_id() == 0) s_i1 = i1;
    }
    __syncthreads();
    const uint64_t i0 = s_i0;
    const uint64_t span = s_i1 - i0 + 1;
    if (span <= T) {
      // stage the tuples; the owners of i0 and i1 have candidates, and so do all the
      // tuples whose slab starts are marked (zero-length slabs share the next start)
      for (uint32_t x = threadIdx.x; x < T; x += kBlock) s_own[x] = 0;
      for (uint32_t t = threadIdx.x; t < span; t += kBlock) {
        const uint64_t i = i0 + t;
        const uint32_t st = (uint32_t)at(i);
        s_start[t] = st;
        if (Q == kJoinSGBase) {
          s_base[t] = R[i];
          s_len[t] = R[i + 1] - R[i] - 1;
          const K inst = dense ? (K)(i >> w) : (K)(b.U[i] >> w);
          s_head[t] = (inst << w) << w;
        } else {
          const K dk = delta[i];
          const uint32_t rb = row_b(i, dk);
          if (Q == kJoinTC) {
            s_head[t] = (dk >> w) << w;
            s_base[t] = rb == kNoRow ? 0u : R[rb];
          } else if (Q == kJoinTri) {
            s_head[t] = dk;
            s_base[t] = rb == kNoRow ? 0u : R[rb];
          } else {
            const uint32_t ra = row_a(i, dk);
            s_head[t] = ((dk >> w) >> w) << w << w;
            const bool live = ra != kNoRow && rb != kNoRow;
            s_aux[t] = live ? R[ra] : 0u;
            s_base[t] = live ? R[rb] : 0u;
            s_len[t] = live ? R[rb + 1] - R[rb] : 1u;
          }
        }
      }
      __syncthreads();
      for (uint32_t t = 1 + threadIdx.x; t < span; t += kBlock) {
        const uint32_t st = s_start[t];
        if (t + 1 == span || s_start[t + 1] != st) s_own[st - (uint32_t)p0] = (uint16_t)t;
      }
      __syncthreads();
      // running max over the marks: position x belongs to the last tuple starting at or before it
      uint32_t own[ITEMS];
      uint32_t mx = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t v = s_own[threadIdx.x * ITEMS + k];
        mx = v > mx ? v : mx;
        own[k] = mx;
      }
      const uint32_t before = block_excl_max(mx, (uint32_t*)s_wave);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        s_own[threadIdx.x * ITEMS + k] = (uint16_t)(own[k] > before ? own[k] : before);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
        if (p < p1) {
          const uint32_t x = (uint32_t)(p - p0);
          const uint32_t t = s_own[x];
          const uint32_t r = (uint32_t)p - s_start[t];
          if (Q == kJoinTC) {
            cand[p] = s_head[t] | (K)Edst[s_base[t] + r];
          } else if (Q == kJoinTri) {
            if (closes(s_head[t], (K)Edst[s_base[t] + r])) ++hits;
          } else if (Q == kJoinSG) {
            const uint32_t lb = s_len[t];
            const uint32_t qa = r / lb;
            const uint32_t rb = r - qa * lb;
            cand[p] = s_head[t] | ((K)Edst[s_aux[t] + qa] << w) | (K)Edst[s_base[t] + rb];
          } else {
            // base rule: ordered pairs (x, y) of distinct children of the row
            const uint32_t len1 = s_len[t];
            const uint32_t qa = r / len1;
            uint32_t qb = r - qa * len1;
            qb += (qb >= qa) ? 1u : 0u;
            cand[p] = s_head[t] | ((K)Edst[s_base[t] + qa] << w) | (K)Edst[s_base[t] + qb];
          }
        }
      }
    } else {
      // more tuples than positions (runs of empty slabs): search each position's tuple
      uint32_t pos[ITEMS];
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
        pos[k] = (uint32_t)min(p, p1 - 1);
      }
      uint64_t li[ITEMS];
      multi_upper_bound_at<ITEMS>([&](uint64_t x) { return (uint32_t)at(i0 + x); }, span, pos, li);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t p = p0 + (uint64_t)k * kBlock + threadIdx.x;
        if (p < p1) {
          const uint64_t i = i0 + li[k] - 1;
          const uint32_t r = (uint32_t)p - (uint32_t)at(i);
          if (Q == kJoinSGBase) {
            const uint32_t len1 = R[i + 1] - R[i] - 1;
            const uint32_t qa = r / len1;
            uint32_t qb = r - qa * len1;
            qb += (qb >= qa) ? 1u : 0u;
            const K inst = dense ? (K)(i >> w) : (K)(b.U[i] >> w);
            cand[p] = ((((inst << w) | (K)Edst[R[i] + qa]) << w) | (K)Edst[R[i] + qb]);
          } else {
            const K dk = delta[i];
            const uint32_t rb = row_b(i, dk);
            if (Q == kJoinTC) {
              cand[p] = ((dk >> w) << w) | (K)Edst[R[rb] + r];
            } else if (Q == kJoinTri) {
              if (closes(dk, (K)Edst[R[rb] + r])) ++hits;
            } else {
              const uint32_t ra = row_a(i, dk);
              const uint32_t lb = R[rb + 1] - R[rb];
              const uint32_t qa = r / lb;
              const uint32_t qb = r - qa * lb;
              const K inst = (dk >> w) >> w;
              cand[p] = ((((inst << w) | (K)Edst[R[ra] + qa]) << w) | (K)Edst[R[rb] + qb]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (Q == kJoinTri) {
    uint64_t total;
    (void)block_excl_scan<uint64_t>(hits, s_wave, total);
    if (threadIdx.x == 0) b.hits[blockIdx.x] = total;
  }
}

// ---------------------------------------------------------------------------
// Hash-join variant of the join (the baseline the paper's binary-search join is
// compared against, Sections III-A and VII): E goes into an open-addressing multimap
// keyed by the source row, built with 64-bit CAS and linear probing; a probe for row b
// walks b's whole cluster.  The count and emit phases are thread-per-tuple, so a hub's
// work is serial in its degree -- the skew the sorted-array join avoids.  A slot holds
// (row << 32 | index of the edge in E); kHashEmpty never equals a stored slot because
// edge indices stay below 2^32 - 16.
// ---------------------------------------------------------------------------
constexpr uint64_t kHashEmpty = ~0ull;

__device__ __forceinline__ uint32_t hash_slot(uint32_t row, uint32_t mask) {
  uint32_t x = row * 0x9E3779B1u;
  x ^= x >> 15;
  x *= 0x85EBCA77u;
  x ^= x >> 13;
  return x & mask;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(uint64_t* __restrict__ a, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
    a[i] = v;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_hash_build(Ctrl* ctrl, Bufs<K> b, int w, uint32_t mask) {
  const uint64_t mu = ctrl->m_unique;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < mu; i += (uint64_t)gridDim.x * kBlock) {
    const uint32_t row = head_row<K>(b.E[i], w);
    const uint64_t entry = ((uint64_t)row << 32) | (uint64_t)i;
    uint32_t slot = hash_slot(row, mask);
    while (atomicCAS((unsigned long long*)&b.htab[slot], (unsigned long long)kHashEmpty,
                     (unsigned long long)entry) != (unsigned long long)kHashEmpty)
      slot = (slot + 1) & mask;
  }
}

// Entries of `row` in the table (walks its cluster to the first empty slot).
__device__ __forceinline__ uint32_t hash_count(const uint64_t* __restrict__ t, uint32_t mask, uint32_t row) {
  uint32_t c = 0;
  for (uint32_t slot = hash_slot(row, mask);; slot = (slot + 1) & mask) {
    const uint64_t e = t[slot];
    if (e == kHashEmpty) return c;
    c += (uint32_t)(e >> 32) == row ? 1u : 0u;
  }
}

template <typename K, int Q, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_join_count_hash(Ctrl* ctrl, Bufs<K> b, int w, uint32_t j,
                                                            uint32_t mask) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint64_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl))) return;
  j = iter_begin(ctrl, j);
  const uint64_t n = b.rec[j - 1].N;
  const K* __restrict__ delta = b.delta[(j - 1) & 1u];
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  const int wid = threadIdx.x / kWave;
  const int lane = lane_id();
  uint64_t running = 0;
  for (uint64_t tbase = lo; tbase < hi; tbase += T) {
    const uint64_t wbase = tbase + (uint64_t)wid * (kWave * ITEMS);
    uint64_t cnt[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t i = wbase + (uint64_t)k * kWave + lane;
      cnt[k] = i < hi ? hash_count(b.htab, mask, tc_join_row<K>(delta[i], w)) : 0u;
    }
    uint64_t ex[ITEMS];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t incl = wave_incl_scan<uint64_t>(cnt[k]);
      ex[k] = run + incl - cnt[k];
      run = sat_add(run, __shfl(incl, kWave - 1, kWave));
    }
    uint64_t tile_total;
    const uint64_t g = block_excl_scan<uint64_t>(lane == 0 ? run : 0ull, s_wave, tile_total);
    const uint64_t wave_base = sat_add(running, __shfl(g, 0, kWave));
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t i = wbase + (uint64_t)k * kWave + lane;
      if (i < hi) b.off[i] = (uint32_t)sat_add(wave_base, ex[k]);
    }
    running = sat_add(running, tile_total);
  }
  if (threadIdx.x == 0) b.jtot[blockIdx.x] = running;
}

// Thread per delta tuple: walk the cluster of its join row again and write every match
// into the tuple's slab (TC), or (kJoinTri) walk the cluster of c for each match (a, c)
// and count the closing edges (c, a).  Same static ranges as the count.
template <typename K, int Q, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_join_emit_hash(Ctrl* ctrl, Bufs<K> b, int w, uint32_t j,
                                                           uint32_t mask) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint64_t s_pre[kScanBlocksMax];
  __shared__ uint64_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl))) return;
  j = iter_cur(ctrl, j);
  const uint64_t n = b.rec[j - 1].N;
  const uint64_t C = block_prefix(b.jtot, gridDim.x, s_pre, s_wave);
  const bool over = Q == kJoinTri ? C > 0xFFFFFFFFull : C > ctrl->cand_cap;
  if (over) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      b.rec[j].C = C;
      atomicOr(&ctrl->overflow, 1u);
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    b.rec[j].C = C;
    ctrl->cand_n = C;
  }
  const K* __restrict__ delta = b.delta[(j - 1) & 1u];
  const uint64_t* __restrict__ t = b.htab;
  const K mask_w = field_mask<K>(w);
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  const uint64_t base = s_pre[blockIdx.x];
  uint64_t hits = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const K dk = delta[i];
    const uint32_t row = tc_join_row<K>(dk, w);
    uint64_t at = base + b.off[i];
    for (uint32_t slot = hash_slot(row, mask);; slot = (slot + 1) & mask) {
      const uint64_t e = t[slot];
      if (e == kHashEmpty) break;
      if ((uint32_t)(e >> 32) != row) continue;
      const K c = (K)b.Edst[(uint32_t)e];
      if (Q == kJoinTri) {
        // closing edge (c, a): walk the cluster of row (inst, c) for destination a
        const K a = (dk >> w) & mask_w;
        const K inst = (dk >> w) >> w;
        const uint32_t rc = (uint32_t)((inst << w) | c);
        for (uint32_t s2 = hash_slot(rc, mask);; s2 = (s2 + 1) & mask) {
          const uint64_t e2 = t[s2];
          if (e2 == kHashEmpty) break;
          if ((uint32_t)(e2 >> 32) == rc && (K)b.Edst[(uint32_t)e2] == a) {
            ++hits;
            break;
          }
        }
      } else {
        b.cand[0][at++] = ((dk >> w) << w) | c;
      }
    }
  }
  if (Q == kJoinTri) {
    __syncthreads();
    uint64_t total;
    (void)block_excl_scan<uint64_t>(hits, s_wave, total);
    if (threadIdx.x == 0) b.hits[blockIdx.x] = total;
  }
}

// ---------------------------------------------------------------------------
// A sort whose input fits one block's LDS (the tail of a fixpoint, small graphs) is done
// by one block in a single launch -- a bitonic network over the keys padded to a power of
// two -- instead of count / scan / scatter launches per pass; the passes then find
// small_sorted set and exit.  Output in the buffer the LSD passes would have ended in.
// The host launches it only where the input may fit (the flag is cleared by the
// compaction that follows every sort, and on resume).
//
// The network runs in registers: thread t holds the keys at positions r * 1024 + t.  A
// compare-exchange between positions jj apart is then inside one thread (jj >= 1024), inside
// one wave (jj < 64: a lane shuffle, no barrier), or through LDS (one store, barrier, load).
// ---------------------------------------------------------------------------
constexpr int kSmallSortThreads = 1024;
static_assert(kSmallJoinTuples == kSmallSortThreads, "the one-block join takes one tuple per thread");

template <typename K>
__device__ __forceinline__ K shfl_xor_key(K v, int lane_mask) {
  if constexpr (sizeof(K) == 4) {
    return (K)(uint32_t)__shfl_xor((int)v, lane_mask, kWave);
  } else {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, lane_mask, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), lane_mask, kWave);
    return ((K)hi << 32) | (K)lo;
  }
}

// The key of lane (this lane ^ M), M a power of two below the wave: a DPP quad permutation
// for M = 1 and 2 (no LDS), a swizzle within 32 lanes for 4, 8 and 16, a permute for 32.
template <int M>
__device__ __forceinline__ uint32_t xor_lanes32(uint32_t v) {
  static_assert(M >= 1 && M <= 32 && (M & (M - 1)) == 0, "");
  if constexpr (M == 1)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1 /* quad_perm 1,0,3,2 */, 0xF, 0xF, false);
  else if constexpr (M == 2)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E /* quad_perm 2,3,0,1 */, 0xF, 0xF, false);
  else if constexpr (M < 32)
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (M << 10) /* and 31, or 0, xor M */);
  else
    return (uint32_t)__shfl_xor((int)v, M, kWave);
}
template <int M, typename K>
__device__ __forceinline__ K xor_lanes(K v) {
  if constexpr (sizeof(K) == 4) {
    return (K)xor_lanes32<M>((uint32_t)v);
  } else {
    const uint32_t lo = xor_lanes32<M>((uint32_t)v);
    const uint32_t hi = xor_lanes32<M>((uint32_t)(v >> 32));
    return ((K)hi << 32) | (K)lo;
  }
}

// Key at position i after its compare-exchange with position i ^ jj (partner key c) in
// the merge of bitonic runs of length k: the lower position keeps the smaller key in an
// ascending run ((i & k) == 0) and the larger one in a descending run.
template <typename K>
__device__ __forceinline__ K bitonic_keep(K a, K c, uint32_t i, uint32_t jj, uint32_t k) {
  const bool take_min = ((i & jj) == 0) == ((i & k) == 0);
  return take_min ? (c < a ? c : a) : (c < a ? a : c);
}

// The compare-exchanges at partner distance M (< one wave) of the merge of bitonic runs of
// length k, for a thread's slots r < E (positions r * kSmallSortThreads + t).
template <int M, typename K, int EMAX>
__device__ __forceinline__ void wave_stage(K (&v)[EMAX], int E, uint32_t k, uint32_t t) {
  if ((uint32_t)M >= k) return;
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    if (r >= E) continue;
    const uint32_t i = (uint32_t)r * kSmallSortThreads + t;
    v[r] = bitonic_keep(v[r], xor_lanes<M>(v[r]), i, (uint32_t)M, k);
  }
}

// Sorts s[0, n) (LDS, n <= CAP) ascending with all kSmallSortThreads threads of the block
// and writes the result to out[0, n) (global; s is clobbered), or with IN_LDS back to
// s[0, n) (out unused; barriers on both sides of the stores).
template <typename K, bool IN_LDS = false, uint32_t CAP = kSmallSortBytes / sizeof(K)>
__device__ __forceinline__ void block_bitonic_sort(K* s, uint32_t n, K* __restrict__ out) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr int EMAX = (int)(CAP / TH);  // keys per thread at most
  const uint32_t t = threadIdx.x;
  uint32_t P = 1;
  while (P < n) P <<= 1;
  const int E = P > TH ? (int)(P / TH) : 1;
  // a wave whose positions are all padding (P below the block) only meets the barriers:
  // the positions below P exchange among themselves (i ^ jj < P for i < P)
  const bool idle = (t & ~(uint32_t)(kWave - 1)) >= P;
  K v[EMAX];
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const uint32_t i = (uint32_t)r * TH + t;
    v[r] = (r < E && i < n) ? s[i] : ~K(0);  // padding sorts last
  }
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t jj = k >> 1; jj >= (uint32_t)kWave; jj >>= 1) {
      if (jj >= TH) {
        // both keys in this thread: slots r and r ^ (jj / TH) (static indices)
#pragma unroll
        for (int rj = 1; rj < EMAX; rj <<= 1) {
          if ((uint32_t)rj * TH != jj) continue;
#pragma unroll
          for (int r = 0; r < EMAX; ++r) {
            if ((r & rj) != 0 || r >= E) continue;
            const uint32_t i = (uint32_t)r * TH + t;
            const K a = v[r], c = v[r | rj];
            const bool asc = (i & k) == 0;
            const K lo = c < a ? c : a, hi = c < a ? a : c;
            v[r] = asc ? lo : hi;
            v[r | rj] = asc ? hi : lo;
          }
        }
      } else if (jj >= (uint32_t)kWave) {
        __syncthreads();  // the previous exchange's loads are done
        if (!idle) {
#pragma unroll
          for (int r = 0; r < EMAX; ++r)
            if (r < E) s[(uint32_t)r * TH + t] = v[r];
        }
        __syncthreads();
        if (!idle) {
#pragma unroll
          for (int r = 0; r < EMAX; ++r) {
            if (r >= E) continue;
            const uint32_t i = (uint32_t)r * TH + t;
            if (i < P) v[r] = bitonic_keep(v[r], s[i ^ jj], i, jj, k);
          }
        }
      }
    }
    // partners within a wave: each distance a constant, no barrier
    if (!idle) {
      wave_stage<32>(v, E, k, t);
      wave_stage<16>(v, E, k, t);
      wave_stage<8>(v, E, k, t);
      wave_stage<4>(v, E, k, t);
      wave_stage<2>(v, E, k, t);
      wave_stage<1>(v, E, k, t);
    }
  }
  if constexpr (IN_LDS) {
    __syncthreads();  // the last exchange through LDS has been read
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
      const uint32_t i = (uint32_t)r * TH + t;
      if (r < E && i < n) s[i] = v[r];
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
      const uint32_t i = (uint32_t)r * TH + t;
      if (r < E && i < n) out[i] = v[r];
    }
  }
}

template <typename K>
__global__ __launch_bounds__(kSmallSortThreads) void k_small_sort(Ctrl* ctrl, const uint64_t* n_ptr,
                                                                  const K* __restrict__ in, K* out,
                                                                  uint32_t alone) {
  constexpr uint32_t CAP = kSmallSortBytes / sizeof(K);
  __shared__ K s[CAP];
  if (block_stop(halted(ctrl))) return;
  const uint64_t n = *n_ptr;
  if (n > CAP) {
    if (threadIdx.x == 0) {
      // no LSD passes follow a sort enqueued alone: halt the loop (the host re-runs the
      // iteration with them)
      if (alone) atomicOr(&ctrl->overflow, 8u);
      else ctrl->small_sorted = 0;
    }
    return;
  }
  for (uint32_t i = threadIdx.x; i < (uint32_t)n; i += kSmallSortThreads) s[i] = in[i];
  __syncthreads();
  block_bitonic_sort<K>(s, (uint32_t)n, out);
  if (threadIdx.x == 0) ctrl->small_sorted = 1;
}

// ---------------------------------------------------------------------------
// One iteration's join and sort in a single block, for the fixpoint's tail (a delta of at
// most kSmallSortThreads tuples whose candidates fit the one-block sort): each thread
// counts one delta tuple's candidates as the count phase does, a block scan lays out the
// slabs, every candidate position finds its tuple by bisection over the slab starts in LDS
// and reads one edge (two for SG), and the candidates are sorted in LDS.  It replaces the
// count, emit and sort launches of such an iteration.  A larger delta or candidate set
// sets overflow bit 3 (halting the loop; the host re-runs the iteration with the
// multi-block launches); the capacity check and the overflow test hook act as in the
// emit phase.
// ---------------------------------------------------------------------------
// Lower / upper bounds of ITEMS keys at once in a sorted LDS array s[0, n) (n < 2^32), the
// first nk of them (nk the same in the whole block), stepping together: 32-bit results,
// for kernels whose registers are tight.
template <typename K, int ITEMS, bool UPPER>
__device__ __forceinline__ void lds_bounds(const K* s, uint32_t n, const K (&v)[ITEMS], uint32_t (&out)[ITEMS],
                                           int nk) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) out[k] = 0;
  if (n == 0) return;
  uint32_t len = n;
  while (len > 1) {
    const uint32_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (k < nk) {
        const K x = s[out[k] + half - 1];
        out[k] = (UPPER ? x <= v[k] : x < v[k]) ? out[k] + half : out[k];
      }
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (k < nk) {
      const K x = s[out[k]];
      out[k] += (UPPER ? x <= v[k] : x < v[k]) ? 1u : 0u;
    }
}
template <typename K, int ITEMS>
__device__ __forceinline__ void lds_lower_bounds(const K* s, uint32_t n, const K (&v)[ITEMS],
                                                 uint32_t (&out)[ITEMS], int nk) {
  lds_bounds<K, ITEMS, false>(s, n, v, out, nk);
}
template <typename K, int ITEMS>
__device__ __forceinline__ void lds_upper_bounds(const K* s, uint32_t n, const K (&v)[ITEMS],
                                                 uint32_t (&out)[ITEMS], int nk) {
  lds_bounds<K, ITEMS, true>(s, n, v, out, nk);
}

// Per-tuple state of a one-block join of at most NT tuples (a multiple of
// kSmallSortThreads), in LDS.
template <typename K, bool SG, uint32_t NT = kSmallSortThreads>
struct OneBlockJoin {
  uint32_t off[NT];           // first candidate
  uint32_t base[NT];          // first edge of the join row
  K head[NT];                 // key bits passed on (SG: the instance)
  uint32_t aux[SG ? NT : 1];  // SG: first edge of the head row
  uint32_t len[SG ? NT : 1];  // SG: length of the join row
};

// Count phase of a one-block join of delta[0, n) (n <= NT; global memory or LDS): thread t
// counts the candidates of tuples [t * NT / kSmallSortThreads, ...) as the count phase
// does and a block scan lays out the slabs.  Returns the candidate total in every thread;
// L.off is complete after the next barrier.
template <typename K, int Q, uint32_t NT = kSmallSortThreads>
__device__ __forceinline__ uint64_t one_block_count(const Ctrl* ctrl, const Bufs<K>& b, int w,
                                                    const K* delta, uint32_t n,
                                                    OneBlockJoin<K, Q == kJoinSG, NT>& L, uint64_t* s_wave) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr uint32_t TUP = NT / TH;  // tuples per thread
  static_assert(NT % TH == 0, "");
  constexpr bool kSG = Q == kJoinSG;
  const bool dense = b.dense != 0;
  const uint32_t* __restrict__ R = b.R;
  uint64_t cs[TUP];
  uint64_t csum = 0;
#pragma unroll
  for (int u = 0; u < (int)TUP; ++u) {
    const uint32_t t = threadIdx.x * TUP + (uint32_t)u;
    uint64_t c = 0;
    if (t < n) {
      const K key = delta[t];
      uint32_t rb = tc_join_row<K>(key, w);
      uint32_t ra = head_row<K>(key, w);
      if (!dense) {
        const uint64_t nu = ctrl->nu;
        const uint64_t jb = lower_bound<uint32_t>(b.U, nu, rb);
        rb = (jb < nu && b.U[jb] == rb) ? (uint32_t)jb : kNoRow;
        if (kSG) {
          const uint64_t ja = lower_bound<uint32_t>(b.U, nu, ra);
          ra = (ja < nu && b.U[ja] == ra) ? (uint32_t)ja : kNoRow;
        }
      }
      if (rb != kNoRow && (!kSG || ra != kNoRow)) {
        const uint32_t base = R[rb];
        const uint32_t lb = R[rb + 1] - base;
        L.base[t] = base;
        if (kSG) {
          const uint32_t aux = R[ra];
          c = (uint64_t)(R[ra + 1] - aux) * lb;
          L.aux[t] = aux;
          L.len[t] = lb;
          L.head[t] = (key >> w) >> w;
        } else {
          c = lb;
          L.head[t] = (key >> w) << w;
        }
      }
    }
    cs[u] = c;
    csum += c;
  }
  uint64_t C;
  uint64_t ex = block_excl_scan<uint64_t, TH / kWave>(csum, s_wave, C);
#pragma unroll
  for (int u = 0; u < (int)TUP; ++u) {
    const uint32_t t = threadIdx.x * TUP + (uint32_t)u;
    if (t < n) L.off[t] = (uint32_t)min<uint64_t>(ex, 0xFFFFFFFFull);
    ex += cs[u];
  }
  return C;
}

// Emit phase of a one-block join counted by one_block_count (C <= the one-block sort's
// capacity): every candidate position finds its tuple by bisection over the slab starts
// and reads one edge (two for SG); the candidates go to s_keys[0, C).  Barriers on both
// sides.
template <typename K, int Q, uint32_t NT = kSmallSortThreads, uint32_t CAP = kSmallSortBytes / sizeof(K)>
__device__ __forceinline__ void one_block_emit(const Bufs<K>& b, int w, uint32_t n, uint32_t C,
                                               const OneBlockJoin<K, Q == kJoinSG, NT>& L, K* s_keys) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr int EMAX = (int)(CAP / TH);
  constexpr bool kSG = Q == kJoinSG;
  const uint32_t t = threadIdx.x;
  const uint32_t* __restrict__ Edst = b.Edst;
  const uint32_t* s_off = L.off;
  const uint32_t* s_base = L.base;
  const K* s_head = L.head;
  const uint32_t* s_aux = L.aux;
  const uint32_t* s_len = L.len;
  __syncthreads();
  // positions r * TH + t: their tuples (the last slab start at or before the position;
  // tuples without candidates share the next start, so the last one holding it has
  // candidates), then every edge load at once
  // (the bisections of all of a thread's positions step together, so their LDS latencies
  // overlap)
  uint32_t e0[EMAX], e1[EMAX], tu[EMAX], pv[EMAX], up[EMAX];
#pragma unroll
  for (int r = 0; r < EMAX; ++r) pv[r] = (uint32_t)r * TH + t;
  lds_upper_bounds<uint32_t, EMAX>(s_off, n, pv, up, (int)((C + TH - 1) / TH));
#pragma unroll
  for (int r = 0; r < EMAX; ++r) tu[r] = pv[r] < C ? up[r] - 1 : 0u;
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const uint32_t p = (uint32_t)r * TH + t;
    if (p < C) {
      const uint32_t u = tu[r];
      const uint32_t q = p - s_off[u];
      if (kSG) {
        const uint32_t lb = s_len[u];
        const uint32_t qa = q / lb;
        e0[r] = Edst[s_aux[u] + qa];
        e1[r] = Edst[s_base[u] + (q - qa * lb)];
      } else {
        e1[r] = Edst[s_base[u] + q];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const uint32_t p = (uint32_t)r * TH + t;
    if (p < C) {
      const K h = s_head[tu[r]];
      s_keys[p] = kSG ? ((((h << w) | (K)e0[r]) << w) | (K)e1[r]) : (h | (K)e1[r]);
    }
  }
  __syncthreads();
}

template <typename K, int Q>
__global__ __launch_bounds__(kSmallSortThreads) void k_small_join(Ctrl* ctrl, Bufs<K> b, int w, uint32_t j,
                                                                  K* __restrict__ out) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr uint32_t CAP = kSmallSortBytes / sizeof(K);
  static_assert(Q == kJoinTC || Q == kJoinSG, "recursive joins only");
  __shared__ K s_keys[CAP];
  __shared__ OneBlockJoin<K, Q == kJoinSG> L;
  __shared__ uint64_t s_wave[TH / kWave];
  if (block_stop(halted(ctrl))) return;
  j = iter_begin(ctrl, j);
  const uint64_t n = b.rec[j - 1].N;
  const uint32_t t = threadIdx.x;
  if (n > TH) {
    if (t == 0) atomicOr(&ctrl->overflow, 8u);
    return;
  }
  const uint64_t C = one_block_count<K, Q>(ctrl, b, w, b.delta[(j - 1) & 1u], (uint32_t)n, L, s_wave);
  const uint32_t hook = ctrl->force_overflow_at;
  if (C > ctrl->cand_cap || (hook != 0 && hook == j)) {
    if (t == 0) {
      b.rec[j].C = C;
      atomicOr(&ctrl->overflow, 1u);
    }
    return;
  }
  if (C > CAP) {
    if (t == 0) {
      b.rec[j].C = C;
      atomicOr(&ctrl->overflow, 8u);
    }
    return;
  }
  if (t == 0) {
    b.rec[j].C = C;
    ctrl->cand_n = C;
  }
  one_block_emit<K, Q>(b, w, (uint32_t)n, (uint32_t)C, L, s_keys);
  block_bitonic_sort<K>(s_keys, (uint32_t)C, out);
}

// ---------------------------------------------------------------------------
// The fixpoint's tail in one launch.  Section V-B keeps the loop on the device and checks
// it from the host once per batch; here, once the delta and an iteration's candidates fit
// one block, a single block runs whole iterations back to back without returning: the
// one-block join and sort above, then dedup and the set difference against Full, then the
// new delta's merge, as the multi-block launches of an iteration do.  Full is A + B + T:
// runs A and B stay as the last multi-block iteration left them (searched through fences
// sampled into LDS, then by bisection in HBM) and the new tuples of the loop gather in a
// sorted run T in LDS (each delta is disjoint from Full, so T's merge is a merge of
// disjoint runs, Section IV-C).  Every iteration writes its delta and its record as the
// multi-block path does; the record's B side is the one the fold after the launch writes
// B + T to (k_tail_fold), and its `tail` field marks it.
//
// The loop ends at the fixpoint or the iteration limit, and leaves the next iteration to
// the multi-block launches when its delta or candidates outgrow one block or could
// overflow the candidate or Full buffers (that path grows them), at the overflow test
// hook, when T could overflow, or past record jmax; ctrl->tail_exit says which.  One block
// of kSmallSortThreads threads, no grid-wide wait.
// ---------------------------------------------------------------------------
constexpr uint32_t kTailFenceBytes = 8192;  // of each of A and B sampled into LDS

// Clears live[k] where v[k] is in either sorted run a[q][0, n[q]) (runs A and B of Full):
// in each run the last of the nf[q] fences (fence f = a[q][f * step[q]], in LDS) at or
// below v[k], then a bisection of the step[q] keys it starts in HBM.  The bisections of
// all keys in both runs step together, so their loads overlap (the dependent round trips
// are those of the longer span only); dead keys load nothing.
template <typename K, int ITEMS>
__device__ __forceinline__ void drop_found(const K* __restrict__ const (&a)[2], const uint64_t (&n)[2], const uint64_t (&step)[2],
                                           const uint32_t (&nf)[2], K (*fence)[kTailFenceBytes / sizeof(K)],
                                           const K (&v)[ITEMS], bool (&live)[ITEMS], int nk) {
  uint64_t pos[2][ITEMS];
  bool act[2][ITEMS];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t f[ITEMS];
    lds_upper_bounds<K, ITEMS>(fence[q], n[q] ? nf[q] : 0u, v, f, nk);  // fences at or below v[k]
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      act[q][k] = k < nk && live[k] && f[k] > 0;  // (below the first fence: below a[q][0])
      pos[q][k] = act[q][k] ? (uint64_t)(f[k] - 1) * step[q] : 0;
    }
  }
  // invariant per run: a[pos] <= v and the last such index lies in [pos, pos + len)
  uint64_t len[2] = {step[0], step[1]};
  while (len[0] > 1 || len[1] > 1) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (len[q] <= 1) continue;
      const uint64_t half = len[q] >> 1;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint64_t x = pos[q][k] + half;
        if (act[q][k] && x < n[q] && a[q][x] <= v[k]) pos[q][k] = x;
      }
      len[q] -= half;
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (act[q][k] && a[q][pos[q][k]] == v[k]) live[k] = false;
}

template <typename K, int Q>
__global__ __launch_bounds__(kSmallSortThreads) void k_tail_loop(Ctrl* ctrl, Bufs<K> b, int w, uint32_t jmax) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr uint32_t CAP = kTailKeys;  // candidates of one iteration
  constexpr uint32_t TCAP = kTailRunBytes / sizeof(K);
  constexpr uint32_t NT = tail_tuples(sizeof(K), Q == kJoinSG);  // delta capacity
  constexpr uint32_t kTailFences = kTailFenceBytes / sizeof(K);
  constexpr int EMAX = (int)(CAP / TH);
  constexpr int TMAX = (int)(TCAP / TH);
  static_assert(Q == kJoinTC || Q == kJoinSG, "recursive joins only");
  __shared__ K s_keys[CAP];                 // the iteration's candidates, then its delta
  __shared__ K s_run[TCAP];                 // T
  __shared__ K s_delta[NT];                 // the delta the next join reads
  __shared__ K s_fence[2][kTailFences];     // samples of A and B
  __shared__ OneBlockJoin<K, Q == kJoinSG, NT> L;
  __shared__ uint64_t s_wave[TH / kWave];
  const uint32_t t = threadIdx.x;
  if (t == 0) ctrl->tail_n = 0;  // (also when halted: the fold after this launch reads it)
  if (block_stop(halted(ctrl))) return;
  uint32_t j = ctrl->iter + 1;
  const IterRec r0 = b.rec[j - 1];
  if (r0.N > NT) {
    if (t == 0) ctrl->tail_exit = kTailSizes;
    return;
  }
  const K* __restrict__ run[2] = {b.full[r0.a], b.fullB[r0.b]};
  const uint64_t rn[2] = {r0.FA, r0.F - r0.FA};
  uint64_t step[2];
  uint32_t nf[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    step[q] = rn[q] > kTailFences ? (rn[q] + kTailFences - 1) / kTailFences : 1;
    nf[q] = (uint32_t)((rn[q] + step[q] - 1) / step[q]);
    for (uint32_t f = t; f < nf[q]; f += TH) s_fence[q][f] = run[q][(uint64_t)f * step[q]];
  }
  uint32_t n = (uint32_t)r0.N;
  for (uint32_t i = t; i < n; i += TH) s_delta[i] = b.delta[(j - 1) & 1u][i];
  const uint64_t cand_cap = ctrl->cand_cap, full_cap = ctrl->full_cap;
  const uint32_t hook = ctrl->force_overflow_at, max_iter = ctrl->max_iter;
  uint64_t F = r0.F;
  uint32_t tn = 0;  // |T|
  uint32_t last = 0;  // the last iteration this launch completed
  uint32_t why = kTailFixpoint;
  __syncthreads();
  for (;; ++j) {
    if (j > jmax) {
      why = kTailRecords;
      break;
    }
    const uint64_t C = one_block_count<K, Q, NT>(ctrl, b, w, s_delta, n, L, s_wave);
    if (C > CAP || C > cand_cap || (hook != 0 && hook == j) || F + C > full_cap) {
      why = kTailSizes;
      break;
    }
    if (tn + C > TCAP) {
      why = kTailRun;
      break;
    }
    one_block_emit<K, Q, NT, CAP>(b, w, n, (uint32_t)C, L, s_keys);
    block_bitonic_sort<K, true, CAP>(s_keys, (uint32_t)C, nullptr);
    // dedup + difference (Section IV-B): thread t takes positions r * TH + t; a key stays
    // if it differs from the key before it and is in none of T, A and B (the searches of
    // all of a thread's keys step together, so their latencies overlap)
    // (rounds r < R hold positions; R is the same in every thread, so the bounds below
    // are scalar branches)
    const int R = (int)((C + TH - 1) / TH);
    K v[EMAX];
    bool live[EMAX];
    uint32_t x[EMAX];
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
      const uint32_t p = (uint32_t)r * TH + t;
      live[r] = r < R && p < C;
      v[r] = live[r] ? s_keys[p] : ~K(0);
      if (live[r] && p > 0 && s_keys[p - 1] == v[r]) live[r] = false;
    }
    lds_lower_bounds<K, EMAX>(s_run, tn, v, x, R);
#pragma unroll
    for (int r = 0; r < EMAX; ++r)
      if (live[r] && x[r] < tn && s_run[x[r]] == v[r]) live[r] = false;
    drop_found<K, EMAX>(run, rn, step, nf, s_fence, v, live, R);
    // output places in position order, (r, t): one block scan of the per-round flags packed
    // into 16-bit fields (four rounds per 64-bit word; a field's sum is at most TH)
    constexpr int W64 = (EMAX + 3) / 4;
    uint64_t packed[W64], before[W64], tot[W64];
#pragma unroll
    for (int q = 0; q < W64; ++q) packed[q] = 0;
#pragma unroll
    for (int r = 0; r < EMAX; ++r) packed[r / 4] |= (uint64_t)(live[r] ? 1u : 0u) << (16 * (r % 4));
#pragma unroll
    for (int q = 0; q < W64; ++q) {
      before[q] = tot[q] = 0;
      if (4 * q < R) before[q] = block_excl_scan<uint64_t, TH / kWave>(packed[q], s_wave, tot[q]);
    }
    // (the scans' barriers order every read of s_keys above before these writes)
    K* __restrict__ dout = b.delta[j & 1u];
    uint32_t N = 0;
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
      const uint32_t o = N + (uint32_t)((before[r / 4] >> (16 * (r % 4))) & 0xFFFFu);
      if (live[r]) {
        s_keys[o] = v[r];
        dout[o] = v[r];
      }
      N += (uint32_t)((tot[r / 4] >> (16 * (r % 4))) & 0xFFFFu);
    }
    __syncthreads();
    // T' = merge(T, delta): every key's place is its index plus its rank in the other run
    K tv[TMAX], dv[EMAX];
    uint32_t tp[TMAX], dp[EMAX];
#pragma unroll
    for (int r = 0; r < TMAX; ++r) {
      const uint32_t i = (uint32_t)r * TH + t;
      tv[r] = i < tn ? s_run[i] : ~K(0);
    }
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
      const uint32_t i = (uint32_t)r * TH + t;
      dv[r] = i < N ? s_keys[i] : ~K(0);
      if (i < N && N <= NT) s_delta[i] = dv[r];
    }
    lds_lower_bounds<K, TMAX>(s_keys, N, tv, tp, (int)((tn + TH - 1) / TH));
    lds_lower_bounds<K, EMAX>(s_run, tn, dv, dp, (int)((N + TH - 1) / TH));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TMAX; ++r) {
      const uint32_t i = (uint32_t)r * TH + t;
      if (i < tn) s_run[i + tp[r]] = tv[r];
    }
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
      const uint32_t i = (uint32_t)r * TH + t;
      if (i < N) s_run[i + dp[r]] = dv[r];
    }
    tn += N;
    const bool at_limit = N > 0 && max_iter != 0 && j >= max_iter;
    if (t == 0) {
      IterRec& rj = b.rec[j];
      rj.N = N;
      rj.C = C;
      rj.F = F + N;
      rj.FA = r0.FA;
      rj.a = r0.a;
      rj.b = tn > 0 ? (r0.b ^ 1u) : r0.b;
      rj.fold = 0;
      rj.tail = 1;
      ctrl->iter = j;
      ctrl->cand_n = C;
      if (N == 0) ctrl->done = 1;
      else if (at_limit) ctrl->limit_hit = 1;
    }
    F += N;
    n = N;
    last = j;
    __syncthreads();  // T and the next delta are in place
    if (N == 0 || at_limit) break;
    if (N > NT) {
      why = kTailSizes;
      break;
    }
  }
  // T goes out for the fold; tn > 0 means at least one iteration completed
  for (uint32_t i = t; i < tn; i += TH) b.tail[i] = s_run[i];
  if (t == 0) {
    if (tn > 0) b.rec[last].tail = 2;
    ctrl->tail_n = tn;
    ctrl->tail_b = r0.b;
    ctrl->tail_exit = why;
    ctrl->full_n = F;
  }
}


// Lanes of the wave (within `active`) whose RB-bit digit equals this lane's: one ballot
// per bit.  For bit b, sb is 0 or all ones (the lane's bit, sign-extended); the lanes that
// agree with this lane on bit b are ballot(bit b) XNOR sb, per 32-lane half.  The ballot
// compares sb itself (so the bit is extracted once) and each half's update
// acc & ~(ballot ^ sb) is one three-input bit operation: four VALU instructions per bit.
// The operation's table is indexed by (first, second, third) operand bits, first most
// significant, so evaluating the function on the patterns 0xF0, 0xCC, 0xAA yields it.
constexpr uint32_t kAndXnor = (0xF0u & ~(0xCCu ^ 0xAAu)) & 0xFFu;  // acc & ~(m ^ sb)
template <int RB>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, uint64_t active) {
  uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
#pragma unroll
  for (int bit = 0; bit < RB; ++bit) {
    const uint32_t sb = (uint32_t)__builtin_amdgcn_sbfe((int)d, bit, 1);
    const uint64_t m = __builtin_amdgcn_uicmp(sb, 0u, 33 /* ICMP_NE */);
    lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)m, sb, kAndXnor);
    hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m >> 32), sb, kAndXnor);
  }
  return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Segmented sort for the TC join.  The emit writes each delta tuple's slab in delta
// order and delta is sorted, so the candidates already come grouped by row (key >> w:
// instance and src) in ascending order; only each row's run needs sorting (by dst).  Block
// b takes tiles of kSegTile positions and owns the runs that start in its tile: it finds
// the first and last run starts in the tile, the end of the run holding the tile's last
// position (the first later position with a larger row, by a wave-parallel search), loads
// that range into LDS, sorts it with the bitonic network above and writes it to `out`.
// Runs partition the array, so every key is written exactly once, and sorting permutes
// keys only inside a run, so rows at every position stay put: in place (out == in) the
// neighbours' searches still read correct rows.
//
// With `long_ok`, a range longer than kSegBitonicMax leaves its last run (the only one
// that can reach past the tile) to k_seg_long: the block sorts the runs before it and
// queues the last one's start and length (three words per row in `queue`, counted in
// ctrl->seg_long).  A run longer than k_seg_long holds, or without `long_ok` a range
// longer than the bitonic network holds, sets overflow bit 4 (halting the loop; the host
// re-runs the iteration with the LSD passes).
// ---------------------------------------------------------------------------
// (a tile a little under 2,048 keeps most ranges -- tile plus the tail of its last run --
// within a 2,048-key network: 2 keys per thread)
constexpr uint32_t kSegTile = 1792;
constexpr uint32_t kSegBitonicMax = 2 * kSegTile;  // longest range sorted by the network
                                                   // when long rows go to k_seg_long
constexpr uint32_t kSegLongBytes = 131072;         // LDS of k_seg_long's row (32K / 16K keys)

template <typename K>
__global__ __launch_bounds__(kSmallSortThreads) void k_seg_sort(int gate, Ctrl* ctrl, const uint64_t* n_ptr,
                                                                const K* in, K* out, int w,
                                                                uint32_t* __restrict__ queue,
                                                                int long_ok) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr uint32_t CAP = kSmallSortBytes / sizeof(K);
  constexpr uint32_t LCAP = kSegLongBytes / sizeof(K);
  static_assert(CAP >= 2 * kSegTile, "a tile and a run reaching past it fit the LDS");
  static_assert(kSegBitonicMax <= CAP, "");
  __shared__ K s[CAP];
  __shared__ uint32_t s_first, s_last;
  __shared__ uint64_t s_end;
  if (block_stop(halted(ctrl) || gated_out(ctrl, gate, kRowMin, kRowFullPerCand))) return;
  const uint64_t n = *n_ptr;
  const uint64_t ntiles = (n + kSegTile - 1) / kSegTile;
  const uint32_t t = threadIdx.x;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t p0 = tile * kSegTile;
    const uint64_t p1 = min<uint64_t>(p0 + kSegTile, n);
    if (t == 0) {
      s_first = kSegTile;
      s_last = 0;
    }
    __syncthreads();
    // run starts in the tile: positions whose row differs from the previous position's
    for (uint32_t q = t; q < (uint32_t)(p1 - p0); q += TH) {
      const uint64_t p = p0 + q;
      if (p == 0 || (in[p] >> w) != (in[p - 1] >> w)) {
        atomicMin(&s_first, q);
        atomicMax(&s_last, q);
      }
    }
    __syncthreads();
    const uint32_t f = s_first;
    if (f < kSegTile && t < (uint32_t)kWave) {
      // end of the run holding p1 - 1: the first position with a larger row, searched up
      // to what one block holds (the network for the whole range; k_seg_long for the run)
      const uint64_t s0 = p0 + f;
      const K last_row = in[p1 - 1] >> w;
      const uint64_t lim = min<uint64_t>(n, long_ok ? p0 + s_last + LCAP : s0 + CAP);
      const uint64_t e = wave_partition(p1, lim, [&](uint64_t i) { return (in[i] >> w) <= last_row; });
      if (t == 0) s_end = (e == lim && lim < n && (in[lim] >> w) == last_row) ? ~0ull : e;
    }
    __syncthreads();
    if (f == kSegTile) continue;  // no run starts here (uniform; s_first is rewritten after
                                  // the barrier that opens the next tile)
    const uint64_t s0 = p0 + f;
    uint64_t e = s_end;
    if (e == ~0ull) {
      if (t == 0) atomicOr(&ctrl->overflow, 16u);
      return;
    }
    if (long_ok && e - s0 > kSegBitonicMax) {
      // the last run goes to k_seg_long; the runs before it lie inside the tile
      const uint64_t sl = p0 + s_last;
      if (t == 0) {
        const uint32_t q = atomicAdd(&ctrl->seg_long, 1u);
        queue[3 * (uint64_t)q] = (uint32_t)sl;
        queue[3 * (uint64_t)q + 1] = (uint32_t)(sl >> 32);
        queue[3 * (uint64_t)q + 2] = (uint32_t)(e - sl);
      }
      e = sl;
    }
    const uint32_t len = (uint32_t)(e - s0);
    for (uint32_t q = t; q < len; q += TH) s[q] = in[s0 + q];
    __syncthreads();
    block_bitonic_sort<K>(s, len, out + s0);
    __syncthreads();
  }
}

// Long rows of the segmented sort: one block per queued row (start, length), the row's
// keys held in LDS and sorted by their dst field (the low w bits; every key of a row has
// the same higher bits) with stable 8-bit LSD passes in LDS, then written to `out` once.
// Each pass ranks as the LSD scatter does: wave `wid` owns a contiguous segment of the
// row, ranks its keys stably by ballots over the digit bits, the per-wave digit counts
// are scanned digit-major into positions, and every key is stored at its position in
// the same LDS array, whose previous contents every wave read into registers before the
// ranking.  A 32-bit-key row of up to 32K keys thus moves through HBM once instead of
// through four global passes and their counts.
template <typename K>
__global__ __launch_bounds__(kSmallSortThreads) void k_seg_long(int gate, Ctrl* ctrl, const K* in, K* out, int w,
                                                                const uint32_t* __restrict__ queue) {
  constexpr uint32_t TH = kSmallSortThreads;
  constexpr int NW = (int)TH / kWave;
  constexpr uint32_t LCAP = kSegLongBytes / sizeof(K);
  constexpr int ITEMS = (int)(LCAP / TH);
  constexpr int RB = 8;
  constexpr int R = 1 << RB;
  static_assert(R <= (int)TH, "one thread per digit");
  __shared__ K s_k[LCAP];
  __shared__ uint32_t s_cnt[NW][R];
  __shared__ uint32_t s_wave[NW];
  if (block_stop(halted(ctrl) || gated_out(ctrl, gate, kRowMin, kRowFullPerCand))) return;
  const uint32_t rows = ctrl->seg_long;
  const int passes = w > RB ? (w + RB - 1) / RB : 1;
  const int tid = threadIdx.x;
  const int wid = tid / kWave;
  const int lane = lane_id();
  const uint64_t lt = lanemask_lt();
  for (uint32_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const uint64_t s0 = (uint64_t)queue[3 * (uint64_t)r] | ((uint64_t)queue[3 * (uint64_t)r + 1] << 32);
    const uint32_t L = queue[3 * (uint64_t)r + 2];
    // wave segments of `seg` keys (a multiple of 64), `kk` per lane
    const uint32_t kk = (L + NW * kWave - 1) / (NW * kWave);
    const uint32_t seg = kk * kWave;
    const uint32_t wofs = (uint32_t)wid * seg;
    K key[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t q = wofs + (uint32_t)k * kWave + lane;
      key[k] = ((uint32_t)k < kk && q < L) ? in[s0 + q] : K(0);
    }
    for (int p = 0; p < passes; ++p) {
      const int shift = p * RB;
      for (int jj = tid; jj < NW * R; jj += TH) (&s_cnt[0][0])[jj] = 0;
      __syncthreads();
      // ranks within the wave's segment (< 2^16), two to a register
      uint32_t rank2[(ITEMS + 1) / 2];
#pragma unroll
      for (int k = 0; k < (ITEMS + 1) / 2; ++k) rank2[k] = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if ((uint32_t)k < kk) {  // uniform
          const bool valid = wofs + (uint32_t)k * kWave + lane < L;
          const uint32_t d = (uint32_t)(key[k] >> shift) & (R - 1);
          const uint64_t active = __builtin_amdgcn_ballot_w64(valid);
          const uint64_t peers = digit_peers<RB>(d, active);
          const uint32_t below = __popcll(peers & lt);
          uint32_t before = 0;
          if (valid) before = s_cnt[wid][d];
          if (valid && below == 0) s_cnt[wid][d] = before + (uint32_t)__popcll(peers);
          rank2[k / 2] |= (before + below) << (16 * (k & 1));
        }
      }
      __syncthreads();
      // digit-major positions: digit base, then the earlier waves' keys of that digit
      uint32_t run = 0;
      if (tid < R) {
#pragma unroll
        for (int v = 0; v < NW; ++v) {
          const uint32_t c = s_cnt[v][tid];
          s_cnt[v][tid] = run;
          run += c;
        }
      }
      uint32_t all;
      const uint32_t base = block_excl_scan<uint32_t, NW>(tid < R ? run : 0u, s_wave, all);
      if (tid < R) {
#pragma unroll
        for (int v = 0; v < NW; ++v) s_cnt[v][tid] += base;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if ((uint32_t)k < kk && wofs + (uint32_t)k * kWave + lane < L) {
          const uint32_t d = (uint32_t)(key[k] >> shift) & (R - 1);
          s_k[s_cnt[wid][d] + ((rank2[k / 2] >> (16 * (k & 1))) & 0xFFFFu)] = key[k];
        }
      }
      __syncthreads();
      if (p + 1 < passes) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          const uint32_t q = wofs + (uint32_t)k * kWave + lane;
          if ((uint32_t)k < kk && q < L) key[k] = s_k[q];
        }
        // (the next pass's first barrier orders these reads before its stores)
      }
    }
    for (uint32_t q = tid; q < L; q += TH) out[s0 + q] = s_k[q];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LSD radix sort (Section V-C): RB bits per pass, dst field first, every pass stable.
//
// A pass is three launches: count (block b counts the digits of a static contiguous
// range of tiles), scan (one block per digit turns the per-block counts into per-block
// offsets) and scatter (block b re-reads its range tile by tile, ranks each tile stably
// in LDS and writes every key to its final position).  Each block writes per-digit runs
// of consecutive positions.  RB is 8 in the paper; wider digits (up to 11 bits) trade
// shorter runs for fewer passes and are picked by the autotuner per key width.
//
// Both range kernels keep the next tile's loads in flight while they work on the current
// one.  A wave whose keys share one digit (common in the passes over the src field,
// whose input is nearly grouped) takes one LDS update instead of RB ballots.
// ---------------------------------------------------------------------------
template <int RB>
struct RadixShape {
  static constexpr int R = 1 << RB;
  // digits owned by each thread for per-digit work: thread t owns [t*DPT, t*DPT+DPT)
  static constexpr int DPT = R >= kBlock ? R / kBlock : 1;
  static constexpr int OWNERS = R >= kBlock ? kBlock : R;
};

// (a whole tile in range loads without per-key bounds checks, which the compiler would
// turn into a branch around every load)
template <typename K, int ITEMS>
__device__ __forceinline__ void load_tile_striped(const K* __restrict__ in, uint64_t base,
                                                  uint64_t hi, K (&key)[ITEMS]) {
  if (base + (uint64_t)ITEMS * kBlock <= hi) {
    const K* p = in + base + threadIdx.x;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) key[k] = p[k * kBlock];
    return;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint64_t i = base + (uint64_t)k * kBlock + threadIdx.x;
    key[k] = i < hi ? in[i] : K(0);
  }
}

// Wave-striped layout of the scatter: wave `wid` owns a contiguous run of 64*ITEMS keys.
template <typename K, int ITEMS>
__device__ __forceinline__ void load_tile_wave(const K* __restrict__ in, uint64_t wbase,
                                               uint64_t hi, K (&key)[ITEMS]) {
  const int lane = lane_id();
  if (wbase + (uint64_t)ITEMS * kWave <= hi) {
    const K* p = in + wbase + lane;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) key[k] = p[k * kWave];
    return;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint64_t i = wbase + (uint64_t)k * kWave + lane;
    key[k] = i < hi ? in[i] : K(0);
  }
}

template <typename K, int RB, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_count(Ctrl* ctrl, const uint64_t* n_ptr,
                                                        const K* __restrict__ in, int shift,
                                                        uint32_t* __restrict__ cnt) {
  using S = RadixShape<RB>;
  constexpr uint32_t T = kBlock * ITEMS;
  // Lanes add into one of COPIES histograms (lane % COPIES), laid out so that the copies
  // of one digit sit in different LDS banks: lanes holding the same digit then collide
  // COPIES times less often.
  constexpr int COPIES = RB <= 8 ? 8 : (RB == 9 ? 4 : (RB == 10 ? 2 : 1));
  constexpr int STRIDE = S::R + 1;
  __shared__ uint32_t s_cnt[COPIES * STRIDE];
  if (block_stop(halted(ctrl) || ctrl->small_sorted)) return;
  const uint64_t n = *n_ptr;
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  if (lo >= hi) return;  // past the active blocks: the scan reads none of their counts
  for (int d = threadIdx.x; d < COPIES * STRIDE; d += kBlock) s_cnt[d] = 0;
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  uint32_t* my = s_cnt + (lane_id() % COPIES) * STRIDE;
  auto count_tile = [&](const K (&key)[ITEMS], uint64_t base, auto full_t) {
    constexpr bool FULL = decltype(full_t)::value;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const bool valid = FULL || base + (uint64_t)k * kBlock + threadIdx.x < hi;
      const uint32_t d = (uint32_t)(key[k] >> shift) & (S::R - 1);
      const uint64_t active = FULL ? ~0ull : __builtin_amdgcn_ballot_w64(valid);
      const uint32_t first = __builtin_amdgcn_readfirstlane(d);
      if (__builtin_amdgcn_ballot_w64(valid && d == first) == active) {
        if (valid && (active & lt) == 0) atomicAdd(&s_cnt[first], (uint32_t)__popcll(active));
      } else if (valid) {
        atomicAdd(&my[d], 1u);
      }
    }
  };
  K cur[ITEMS];
  load_tile_striped<K, ITEMS>(in, lo, hi, cur);
  for (uint64_t base = lo; base < hi; base += T) {
    K nxt[ITEMS];
    if (base + T < hi) load_tile_striped<K, ITEMS>(in, base + T, hi, nxt);
    if (base + T <= hi) count_tile(cur, base, std::true_type());
    else count_tile(cur, base, std::false_type());
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) cur[k] = nxt[k];
  }
  __syncthreads();
  for (int d = threadIdx.x; d < S::R; d += kBlock) {
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < COPIES; ++r) c += s_cnt[r * STRIDE + d];
    cnt[(uint64_t)d * gridDim.x + blockIdx.x] = c;
  }
}

// One block per digit: per-block counts of the digit -> exclusive per-block offsets (in
// place); tot[d] = the digit's total.  Only the blocks that own keys wrote counts.
__global__ __launch_bounds__(kBlock) void k_radix_scan(Ctrl* ctrl, const uint64_t* n_ptr, uint32_t T,
                                                       uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ tot, int G) {
  __shared__ uint32_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl) || ctrl->small_sorted)) return;
  const int GA = (int)active_blocks(*n_ptr, T, (uint32_t)G);
  uint32_t* row = cnt + (uint64_t)blockIdx.x * G;
  uint32_t carry = 0;
  for (int base = 0; base < GA; base += kBlock) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < GA ? row[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<uint32_t>(v, s_wave, total);
    if (i < GA) row[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Digit peers through a per-wave LDS table instead of RB ballots (digits of up to 9 bits,
// where the table is small): every lane sets its lane bit in the entry of its digit (one
// LDS atomic OR into the entry's half for its 32-lane half), reads the whole entry back --
// the mask of the lanes holding the same digit -- and the lowest such lane clears the entry
// for the next key.  LDS instructions of one wave execute in order, so every OR of an
// instruction lands before the reads of the next and every read before the clear.  About
// a dozen VALU instructions per key against four per digit bit for the ballots.
template <int RB>
struct PeerTable {
  static constexpr bool kOn = RB <= 9;
  static constexpr int kWords = kOn ? 2 * (1 << RB) : 1;  // per wave: low halves, then high
};

template <typename K, int RB, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(Ctrl* ctrl, const uint64_t* n_ptr,
                                                          const K* __restrict__ in,
                                                          K* __restrict__ out, int shift,
                                                          const uint32_t* __restrict__ off,
                                                          const uint32_t* __restrict__ tot) {
  using S = RadixShape<RB>;
  using PT = PeerTable<RB>;
  constexpr int DPT = S::DPT;
  constexpr uint32_t T = kBlock * ITEMS;
  static_assert(T <= 65535, "tile offsets are kept in 16 bits");
  __shared__ K s_keys[T];
  __shared__ uint16_t s_cnt[kWavesPerBlock][S::R];  // per-wave digit counts, then offsets
  __shared__ uint16_t s_loc[S::R];                  // first tile position of each digit
  __shared__ uint32_t s_run[S::R];                  // next output position of each digit
  __shared__ uint32_t s_wave[kWavesPerBlock];
  __shared__ uint32_t s_peer[kWavesPerBlock * PT::kWords];  // peer table of each wave
  if (block_stop(halted(ctrl) || ctrl->small_sorted)) return;
  const uint64_t n = *n_ptr;
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  if (lo >= hi) return;
  const int tid = threadIdx.x;
  const int wid = tid / kWave;
  const int lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const bool owner = tid < S::OWNERS;
  uint32_t* const peer_lo = s_peer + wid * PT::kWords;  // entry d: lanes 0..31 at [d], 32..63 at [R + d]
  const uint32_t peer_bit = 1u << (lane & 31);
  const uint32_t peer_half = lane >= 32 ? (uint32_t)S::R : 0u;
  if (PT::kOn)
    for (int jj = tid; jj < kWavesPerBlock * PT::kWords; jj += kBlock) s_peer[jj] = 0;  // (before the
                                                                                        // barrier below)
  {
    // first position of each digit for this block: digit base + earlier blocks' keys
    uint32_t t[DPT];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      t[i] = owner ? tot[tid * DPT + i] : 0u;
      sum += t[i];
    }
    uint32_t all;
    uint32_t base = block_excl_scan<uint32_t>(sum, s_wave, all);
    if (owner) {
#pragma unroll
      for (int i = 0; i < DPT; ++i) {
        const int d = tid * DPT + i;
        s_run[d] = base + off[(uint64_t)d * gridDim.x + blockIdx.x];
        base += t[i];
      }
    }
  }
  // One tile: stable rank in LDS, then every key to its final position.  FULL tiles (all
  // but possibly the last of the range) skip the per-key bounds checks.
  auto scatter_tile = [&](const K (&cur)[ITEMS], uint64_t tbase, auto full_t) {
    constexpr bool FULL = decltype(full_t)::value;
    for (int jj = tid; jj < kWavesPerBlock * S::R; jj += kBlock) (&s_cnt[0][0])[jj] = 0;
    __syncthreads();
    // wave-striped: wave `wid` owns a contiguous run of 64*ITEMS keys
    const uint32_t wofs = (uint32_t)wid * (ITEMS * kWave);
    const uint32_t tile_n = FULL ? T : (uint32_t)(hi - tbase);
    uint32_t rank[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const bool valid = FULL || wofs + (uint32_t)k * kWave + lane < tile_n;
      const uint32_t d = (uint32_t)(cur[k] >> shift) & (S::R - 1);
      const uint64_t active = FULL ? ~0ull : __builtin_amdgcn_ballot_w64(valid);
      const uint32_t first = __builtin_amdgcn_readfirstlane(d);
      if (__builtin_amdgcn_ballot_w64(valid && d == first) == active) {
        // every active lane holds digit `first`
        const uint32_t before = s_cnt[wid][first];
        rank[k] = before + (uint32_t)__popcll(active & lt);
        if (valid && (active & lt) == 0) s_cnt[wid][first] = (uint16_t)(before + __popcll(active));
      } else if (PT::kOn) {
        uint64_t peers = 0;
        uint32_t before = 0;
        if (valid) {
          atomicOr(&peer_lo[peer_half + d], peer_bit);
          peers = ((uint64_t)peer_lo[S::R + d] << 32) | peer_lo[d];
          before = s_cnt[wid][d];
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        if (valid && below == 0) {
          s_cnt[wid][d] = (uint16_t)(before + __popcll(peers));
          peer_lo[d] = 0u;
          peer_lo[S::R + d] = 0u;
        }
        rank[k] = before + below;
      } else {
        const uint64_t peers = digit_peers<RB>(d, active);
        const uint32_t below = __popcll(peers & lt);
        uint32_t before = 0;
        if (valid) before = s_cnt[wid][d];
        if (valid && below == 0) s_cnt[wid][d] = (uint16_t)(before + __popcll(peers));
        rank[k] = before + below;
      }
    }
    __syncthreads();
    // owned digits: per-wave exclusive offsets, tile totals, tile-local digit starts
    uint32_t tile_cnt[DPT];
    uint32_t own_sum = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = tid * DPT + i;
      uint32_t c_run = 0;
      if (owner) {
#pragma unroll
        for (int w2 = 0; w2 < kWavesPerBlock; ++w2) {
          const uint32_t c = s_cnt[w2][d];
          s_cnt[w2][d] = (uint16_t)c_run;
          c_run += c;
        }
      }
      tile_cnt[i] = c_run;
      own_sum += c_run;
    }
    uint32_t total;
    uint32_t start = block_excl_scan<uint32_t>(own_sum, s_wave, total);
    if (owner) {
#pragma unroll
      for (int i = 0; i < DPT; ++i) {
        s_loc[tid * DPT + i] = (uint16_t)start;
        start += tile_cnt[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      if (FULL || wofs + (uint32_t)k * kWave + lane < tile_n) {
        const uint32_t d = (uint32_t)(cur[k] >> shift) & (S::R - 1);
        const uint32_t pos = (uint32_t)s_loc[d] + s_cnt[wid][d] + rank[k];
        if (FULL || pos < T) s_keys[pos] = cur[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t jj = (uint32_t)k * kBlock + tid;
      if (FULL || jj < tile_n) {
        const K kk = s_keys[jj];
        const uint32_t d = (uint32_t)(kk >> shift) & (S::R - 1);
        const uint32_t pos = s_run[d] + (jj - s_loc[d]);  // < n < 2^32
        if (FULL || pos < n) out[pos] = kk;
      }
    }
    __syncthreads();
    if (owner) {
#pragma unroll
      for (int i = 0; i < DPT; ++i) s_run[tid * DPT + i] += tile_cnt[i];
    }
  };
  K cur[ITEMS];
  load_tile_wave<K, ITEMS>(in, lo + (uint64_t)wid * (ITEMS * kWave), hi, cur);
  for (uint64_t tbase = lo; tbase < hi; tbase += T) {
    K nxt[ITEMS];
    if (tbase + T < hi) load_tile_wave<K, ITEMS>(in, tbase + T + (uint64_t)wid * (ITEMS * kWave), hi, nxt);
    if (tbase + T <= hi) scatter_tile(cur, tbase, std::true_type());
    else scatter_tile(cur, tbase, std::false_type());
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) cur[k] = nxt[k];
  }
}

// ---------------------------------------------------------------------------
// Compaction: fused dedup + set difference (Section IV-B), also used for seeding the
// relations (dedup only) and for the SG diagonal filter.
//
// compact_local: block b owns a static range of the sorted input.  A key survives dedup
// when it is the first of its run of equal keys (the key before the range is read from
// memory) and, in iteration mode, is absent from Full.  For each tile the window of Full
// that can hold its keys is found by two wave-parallel searches inside the block's own
// Full range; a window of at most a tile is staged in LDS and searched there, a larger
// one through every st-th key staged in LDS, then in place.  Survivors are
// compacted, in input order, to the start of the block's range in a scratch buffer.
//
// compact_gather: every block adds up the survivor counts of the blocks before it and
// copies its survivors to their final positions; the output stays sorted.  Block 0 then
// records the iteration (|Delta^j|, |Full| after it, the fixpoint and limit flags).
// ---------------------------------------------------------------------------
// keep[k] = false for every item of this thread present in the sorted LDS window w[0, n)
// (n >= 1).  The thread's items are ascending: two bisections (in lockstep) bound the
// part of the window they can hit, then every item bisects that part independently, all
// items in lockstep, so the LDS reads of one step overlap instead of forming a chain.
template <typename K, int ITEMS>
__device__ __forceinline__ void drop_present(const K* w, uint32_t n, const K (&cv)[ITEMS],
                                             bool (&keep)[ITEMS]) {
  uint32_t lo = 0, hi = 0;
  for (uint32_t len = n; len > 1;) {
    const uint32_t half = len >> 1;
    lo = (w[lo + half - 1] < cv[0]) ? lo + half : lo;
    hi = (w[hi + half - 1] <= cv[ITEMS - 1]) ? hi + half : hi;
    len -= half;
  }
  lo += (w[lo] < cv[0]) ? 1u : 0u;
  hi += (w[hi] <= cv[ITEMS - 1]) ? 1u : 0u;
  if (hi <= lo) return;
  uint32_t p[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) p[k] = lo;
  for (uint32_t len = hi - lo; len > 1;) {
    const uint32_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) p[k] = (w[p[k] + half - 1] < cv[k]) ? p[k] + half : p[k];
    len -= half;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t q = p[k] + ((w[p[k]] < cv[k]) ? 1u : 0u);
    if (q < hi && w[q] == cv[k]) keep[k] = false;
  }
}

// The same for a window g[0, gn) too large for LDS: `s` holds every st-th key of it
// (s[i] = g[i * st], ns entries).  Each item finds its stretch of st keys among the
// samples (LDS), then bisects that stretch in place; all items in lockstep.
template <typename K, int ITEMS>
__device__ __forceinline__ void drop_present_sampled(const K* s, uint32_t ns, const K* __restrict__ g,
                                                     uint32_t gn, uint32_t st, const K (&cv)[ITEMS],
                                                     bool (&keep)[ITEMS]) {
  uint32_t u[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) u[k] = 0;
  for (uint32_t len = ns; len > 1;) {
    const uint32_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) u[k] = (s[u[k] + half - 1] <= cv[k]) ? u[k] + half : u[k];
    len -= half;
  }
  uint32_t p[ITEMS], end[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    u[k] += (s[u[k]] <= cv[k]) ? 1u : 0u;  // samples <= the item
    p[k] = u[k] ? (u[k] - 1) * st : 0u;
    end[k] = u[k] ? min(p[k] + st, gn) : 1u;
  }
  // reads past a stretch's end are clamped to its last key (as if +infinity: when that
  // key is below the item the item is absent either way)
  for (uint32_t len = st; len > 1;) {
    const uint32_t half = len >> 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t at = min(p[k] + half - 1, end[k] - 1);
      p[k] = (g[at] < cv[k]) ? p[k] + half : p[k];
    }
    len -= half;
  }
  // the item is at p or p + 1 if present: both keys are loaded at once
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const K x0 = g[min(p[k], end[k] - 1)];
    const K x1 = g[min(p[k] + 1, end[k] - 1)];
    const bool past = x0 < cv[k];
    const uint32_t q = p[k] + (past ? 1u : 0u);
    if (u[k] && q < end[k] && (past ? x1 : x0) == cv[k]) keep[k] = false;
  }
}

// Items per block range of the compaction.  At least a tile per block: whole tiles.  A
// smaller input is spread evenly over the grid (down to one key per block), so that each
// block's windows of Full are about 1/G of it: staged whole in LDS where a tile's window
// of a large input needs dependent searches in place.  The local and gather launches use
// the same grid, hence the same ranges.
__device__ __forceinline__ uint32_t compact_span(uint64_t n, uint32_t T, uint32_t G) {
  const uint64_t per = (n + G - 1) / G;
  if (per >= T) return T;
  return per > 1 ? (uint32_t)per : 1u;
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_compact_local(Ctrl* ctrl, int mode, const uint64_t* n_ptr,
                                                          const K* __restrict__ in,
                                                          K* __restrict__ tmp, Bufs<K> b, int w,
                                                          uint32_t j) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_c[T + 1];
  __shared__ K s_f[2 * T];  // windows of A [0, T) and B [T, 2T); then the survivors
  __shared__ uint32_t s_wave[kWavesPerBlock];
  __shared__ uint64_t s_lo[2], s_hi[2];
  const bool filt = (mode & kModeFilter) != 0;
  if (block_stop((!filt && halted(ctrl)) ||
                 gated_out(ctrl, (mode & kModeGateRow) ? 1 : ((mode & kModeGateSort) ? 2 : 0), kRowMin,
                           kRowFullPerCand)))
    return;
  j = iter_cur(ctrl, j);
  const uint64_t n = *n_ptr;
  uint64_t lo, hi;
  block_range(n, compact_span(n, T, gridDim.x), lo, hi);
  if (lo >= hi) {
    if (threadIdx.x == 0) b.bcnt[blockIdx.x] = 0;
    return;
  }
  // the first tile's keys are loaded now, so their latency overlaps the searches below
  K first[ITEMS];
  {
    const uint32_t tn0 = (uint32_t)min<uint64_t>(T, hi - lo);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t jj = (uint32_t)k * kBlock + threadIdx.x;
      first[k] = jj < tn0 ? in[lo + jj] : K(0);
    }
  }
  const K before_lo = (threadIdx.x == 0 && lo > 0) ? in[lo - 1] : K(0);
  const bool diff = (mode & kModeIter) != 0;
  // Full of iteration j-1: runs A and B, each tile's window of each staged in LDS when it
  // fits (searched in place otherwise)
  const K* __restrict__ runA = nullptr;
  const K* __restrict__ runB = nullptr;
  uint64_t FA = 0, FB = 0;
  if (diff) {
    const IterRec rp = b.rec[j - 1];
    runA = b.full[rp.a];
    runB = b.fullB[rp.b];
    FA = rp.FA;
    FB = rp.F - rp.FA;
  }
  const K mask = field_mask<K>(w);
  const int wid = threadIdx.x / kWave;
  // the parts of A and B that can hold any key of this block (four waves search at once)
  uint64_t alo = 0, ahi = 0, blo = 0, bhi = 0;
  if (diff) {
    if (wid == 0) {
      const uint64_t v = wave_lower_bound(runA, FA, in[lo]);
      if (lane_id() == 0) s_lo[0] = v;
    } else if (wid == 1) {
      const uint64_t v = wave_upper_bound(runA, FA, in[hi - 1]);
      if (lane_id() == 0) s_hi[0] = v;
    } else if (wid == 2) {
      const uint64_t v = wave_lower_bound(runB, FB, in[lo]);
      if (lane_id() == 0) s_lo[1] = v;
    } else {
      const uint64_t v = wave_upper_bound(runB, FB, in[hi - 1]);
      if (lane_id() == 0) s_hi[1] = v;
    }
    __syncthreads();
    alo = s_lo[0];
    ahi = s_hi[0] > alo ? s_hi[0] : alo;
    blo = s_lo[1];
    bhi = s_hi[1] > blo ? s_hi[1] : blo;
    __syncthreads();
  }
  uint64_t running = 0;
  // each tile's windows start where the previous tile's ended (tiles are consecutive keys):
  // only the ends are searched, from the current starts
  uint64_t a_at = alo, b_at = blo;
  for (uint64_t tbase = lo; tbase < hi; tbase += T) {
    const uint32_t tn = (uint32_t)min<uint64_t>(T, hi - tbase);
    if (tbase == lo) {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t jj = (uint32_t)k * kBlock + threadIdx.x;
        if (jj < tn) s_c[jj + 1] = first[k];
      }
      if (threadIdx.x == 0 && tbase > 0) s_c[0] = before_lo;
    } else {
      for (uint32_t jj = threadIdx.x; jj < tn; jj += kBlock) s_c[jj + 1] = in[tbase + jj];
      if (threadIdx.x == 0) s_c[0] = in[tbase - 1];
    }
    if (diff) {
      // ends of the windows of A and B that can hold this tile's keys (the last tile's
      // are the ends of the block's parts, found above)
      const K last = in[tbase + tn - 1];
      if (tbase + tn >= hi) {
        if (threadIdx.x == 0) {
          s_hi[0] = ahi;
          s_hi[1] = bhi;
        }
      } else if (wid == 0) {
        const uint64_t v = a_at + wave_upper_bound(runA + a_at, ahi - a_at, last);
        if (lane_id() == 0) s_hi[0] = v;
      } else if (wid == 1) {
        const uint64_t v = b_at + wave_upper_bound(runB + b_at, bhi - b_at, last);
        if (lane_id() == 0) s_hi[1] = v;
      }
    }
    __syncthreads();
    uint64_t flo = 0, fspan = 0, glo = 0, gspan = 0;
    bool win = false, gwin = false;
    uint32_t fst = 1, gst = 1;
    if (diff) {
      const uint64_t a_end = s_hi[0], b_end = s_hi[1];
      flo = a_at;
      fspan = a_end - a_at;
      glo = b_at;
      gspan = b_end - b_at;
      // the next tile's first key may equal this tile's last, and so the last key of a
      // window: then the next window starts one earlier
      if (tbase + tn < hi) {
        const K next = in[tbase + tn];
        a_at = (a_end > a_at && runA[a_end - 1] == next) ? a_end - 1 : a_end;
        b_at = (b_end > b_at && runB[b_end - 1] == next) ? b_end - 1 : b_end;
      }
      win = fspan <= T;
      gwin = gspan <= T;
      // a window that fits is staged whole, a larger one as every st-th key
      fst = win ? 1u : (uint32_t)((fspan + T - 1) / T);
      gst = gwin ? 1u : (uint32_t)((gspan + T - 1) / T);
      const uint32_t fns = (uint32_t)((fspan + fst - 1) / fst);
      const uint32_t gns = (uint32_t)((gspan + gst - 1) / gst);
      for (uint32_t jj = threadIdx.x; jj < fns; jj += kBlock) s_f[jj] = runA[flo + (uint64_t)jj * fst];
      for (uint32_t jj = threadIdx.x; jj < gns; jj += kBlock) s_f[T + jj] = runB[glo + (uint64_t)jj * gst];
      __syncthreads();
    }
    const uint32_t j0 = threadIdx.x * ITEMS;
    K cv[ITEMS];
    bool keep[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t jj = j0 + k;
      // past the tile: the largest key keeps the thread's items ascending (never kept)
      cv[k] = (jj < tn) ? s_c[jj + 1] : ~K(0);
      if (filt) keep[k] = jj < tn && ((cv[k] >> w) & mask) != (cv[k] & mask);
      else keep[k] = jj < tn && ((tbase + jj == 0) || (cv[k] != s_c[jj]));
    }
    if (fspan > 0) {
      if (win) {
        drop_present<K, ITEMS>(s_f, (uint32_t)fspan, cv, keep);
      } else {
        drop_present_sampled<K, ITEMS>(s_f, (uint32_t)((fspan + fst - 1) / fst), runA + flo, (uint32_t)fspan,
                                       fst, cv, keep);
      }
    }
    if (gspan > 0) {
      if (gwin) {
        drop_present<K, ITEMS>(s_f + T, (uint32_t)gspan, cv, keep);
      } else {
        drop_present_sampled<K, ITEMS>(s_f + T, (uint32_t)((gspan + gst - 1) / gst), runB + glo,
                                       (uint32_t)gspan, gst, cv, keep);
      }
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) cnt += keep[k] ? 1u : 0u;
    uint32_t tile_total;
    const uint32_t ex = block_excl_scan<uint32_t>(cnt, s_wave, tile_total);
    // (the scan ends with a barrier, so s_f is free for the survivors)
    uint32_t lpos = (uint32_t)ex;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (keep[k]) s_f[lpos++] = cv[k];
    __syncthreads();
    for (uint32_t jj = threadIdx.x; jj < (uint32_t)tile_total; jj += kBlock)
      tmp[lo + running + jj] = s_f[jj];
    running += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) b.bcnt[blockIdx.x] = running;
}

// ---------------------------------------------------------------------------
// Row-bitmap sort + dedup + set difference (TC, ids of at most kRowBitsMax bits): the
// segmented dst-only sort of Section V-C carried through the difference of Section IV-B.
// The join writes each delta tuple's slab in delta order and the delta is sorted, so the
// candidates come grouped by row (key >> w: instance and src) in ascending row order; only
// their order within a row is open.  A row's keys share their upper bits, so the row is a
// set of at most 2^w dst values: one bit each in an LDS bitmap.  Block b owns the rows
// that start in its static range of positions.  For each row it streams the row's
// candidates into one bitmap (LDS atomic OR: duplicates collapse), the row's keys of Full
// runs A and B into another, and writes the bits of cand & ~full in bit order -- the row's
// new tuples, sorted and duplicate-free -- one survivor per thread and step, so writes
// coalesce.  Full's cursors advance with the rows (a row's keys of A and B are contiguous
// and rows ascend); a row not right after the previous one is found by a wave search.
// Survivors go to tmp from the block's first row start on (its rows' candidate span, which
// no other block's span overlaps), counted in bcnt with the start in bstart, for the
// gather.  This replaces the LSD passes and the compaction of such an iteration with one
// streaming pass over its candidates and the rows of Full they touch.
// ---------------------------------------------------------------------------
constexpr uint32_t kRowWordsMax = (1u << kRowBitsMax) / 32;
constexpr int kRowItems = 4;                      // keys per thread per round
constexpr uint32_t kRowTile = kBlock * kRowItems;  // keys streamed per round

// Position of the k-th set bit (k = 0 the lowest) of v, which has more than k set bits.
__device__ __forceinline__ uint32_t nth_set_bit(uint32_t v, uint32_t k) {
  uint32_t pos = 0;
  uint32_t c = (uint32_t)__popc(v & 0xFFFFu);
  if (k >= c) { k -= c; v >>= 16; pos += 16; }
  c = (uint32_t)__popc(v & 0xFFu);
  if (k >= c) { k -= c; v >>= 8; pos += 8; }
  c = (uint32_t)__popc(v & 0xFu);
  if (k >= c) { k -= c; v >>= 4; pos += 4; }
  c = (uint32_t)__popc(v & 0x3u);
  if (k >= c) { k -= c; v >>= 2; pos += 2; }
  if (k >= (v & 1u)) pos += 1;
  return pos;
}

// Set the bits of sorted, distinct keys held by consecutive lanes (bit d of bm for every
// lane with `valid`): the lanes of one word form a run of at most 32, whose bits a shuffle
// scan gathers into its last lane, which alone writes -- one LDS atomic per word instead
// of up to 32 queued on one address (a row of Full late in a fixpoint is long runs of
// consecutive ids).
__device__ __forceinline__ void or_sorted_runs(uint32_t* bm, bool valid, uint32_t d) {
  const int lane = lane_id();
  const uint32_t word = valid ? (d >> 5) : 0xFFFFFFFFu;
  uint32_t acc = valid ? (1u << (d & 31u)) : 0u;
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) {
    const uint32_t o = __shfl_up(acc, off, kWave);
    const uint32_t ow = __shfl_up(word, off, kWave);
    if (lane >= off && ow == word) acc |= o;
  }
  const uint32_t next = __shfl_down(word, 1, kWave);
  if (valid && (lane == kWave - 1 || next != word)) atomicOr(&bm[word], acc);
}

// The row pass's searches (its rows' range, Full's cursors): rounds of kRowFan probes until
// the span fits one 64-lane round (0: every round 64 probes).  A round of 64 probes touches
// 64 scattered lines; thousands of blocks search at their start.
constexpr int kRowFan = 8;
template <typename Pred>
__device__ __forceinline__ uint64_t row_search(uint64_t lo, uint64_t hi, Pred pred) {
  if constexpr (kRowFan > 0)
    return wave_partition_fan<kRowFan>(lo, hi, pred);
  else
    return wave_partition(lo, hi, pred);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_row_diff(int gate, Ctrl* ctrl, const uint64_t* n_ptr,
                                                     const K* __restrict__ in, K* __restrict__ tmp, Bufs<K> b,
                                                     int w, uint32_t j) {
  __shared__ uint32_t s_cb[kRowWordsMax];   // the row's candidate bits, then its new bits
  __shared__ uint32_t s_fb[kRowWordsMax];   // the row's bits of Full
  __shared__ uint32_t s_pre[kRowWordsMax];  // new bits in the words before each word
  __shared__ uint32_t s_wave[kWavesPerBlock];
  __shared__ uint64_t s_at[3];              // broadcast of wave searches
  if (block_stop(halted(ctrl) || gated_out(ctrl, gate, kRowMin, kRowFullPerCand))) return;
  // this iteration needs no sort: LSD passes enqueued behind (the other route) are no-ops
  // (the gather clears the flag)
  if (gate != 0 && blockIdx.x == 0 && threadIdx.x == 0) ctrl->small_sorted = 1;
  j = iter_cur(ctrl, j);
  const uint64_t n = *n_ptr;
  const uint32_t tid = threadIdx.x;
  const int wid = (int)(tid / kWave);
  const IterRec rp = b.rec[j - 1];
  const K* __restrict__ runA = b.full[rp.a];
  const K* __restrict__ runB = b.fullB[rp.b];
  const uint64_t FA = rp.FA, FB = rp.F - rp.FA;
  // Rows for this block: a row costs its candidates and its keys of Full, so the blocks
  // split the rows by rank in the merge (by row) of the candidates and the larger run of
  // Full -- equal shares of both -- rather than by candidate position alone.  Block b owns
  // the rows from the row at merged rank b*T/G up to the one at rank (b+1)*T/G; a row
  // spanning several boundaries goes to the last block whose boundary falls in it.
  {
    const bool xa = FA >= FB;
    const K* __restrict__ X = xa ? runA : runB;
    const uint64_t nx = xa ? FA : FB;
    const uint64_t total = n + nx;
    constexpr uint64_t kInf = ~0ull;
    // row of the element at merged rank d (rows of Full first on ties); kInf past the end
    auto row_at = [&](uint64_t d) -> uint64_t {
      if (d >= total) return kInf;
      const uint64_t ilo = d > nx ? d - nx : 0, ihi = d < n ? d : n;
      // candidates among the first d merged elements: C[i] precedes X[d-1-i] while its row
      // is smaller (true for a prefix of i)
      const uint64_t i = row_search(ilo, ihi, [&](uint64_t q) {
        return (uint64_t)(in[q] >> w) < (uint64_t)(X[d - 1 - q] >> w);
      });
      const uint64_t rc = i < n ? (uint64_t)(in[i] >> w) : kInf;
      const uint64_t rx = d - i < nx ? (uint64_t)(X[d - i] >> w) : kInf;
      return rc < rx ? rc : rx;
    };
    // first candidate position whose row is at least r
    auto row_pos = [&](uint64_t r) -> uint64_t {
      if (r == kInf) return n;
      return row_search(0, n, [&](uint64_t q) { return (uint64_t)(in[q] >> w) < r; });
    };
    if (wid < 2) {
      const uint64_t d = (total * (uint64_t)(blockIdx.x + wid)) / gridDim.x;
      const uint64_t v = row_pos(blockIdx.x + wid == 0 ? 0 : row_at(d));
      if (lane_id() == 0) s_at[wid] = v;
    }
    __syncthreads();
  }
  const uint64_t lo = s_at[0], hi = s_at[1];
  __syncthreads();
  uint64_t p = lo;
  const uint64_t out0 = p;
  uint64_t running = 0;
  if (p < hi) {
    const uint32_t words = w > 5 ? 1u << (w - 5) : 1u;
    const K fmask = field_mask<K>(w);
    // Full's cursors at the first row's keys
    {
      const K first = (in[p] >> w) << w;
      if (wid == 0) {
        const uint64_t v = row_search(0, FA, [&](uint64_t i) { return runA[i] < first; });
        if (lane_id() == 0) s_at[1] = v;
      } else if (wid == 1) {
        const uint64_t v = row_search(0, FB, [&](uint64_t i) { return runB[i] < first; });
        if (lane_id() == 0) s_at[2] = v;
      }
      __syncthreads();
    }
    uint64_t pa = s_at[1], pb = s_at[2];
    // Set the bits of row rk's keys in X[from, nx) into bm, tile by tile; returns the position
    // past them.  Rows ascend and X[from] is the row's first key or later, so in every tile
    // the row's keys are a prefix: the row ends where a tile holds fewer than it could.
    // `check`: a key whose bit is already set in s_fb or bm (a duplicate, or a tuple of
    // Full) skips the atomic -- a plain LDS read, which lanes of one word share.
    auto stream_row = [&](const K* __restrict__ X, uint64_t nx, uint64_t from, K rk, uint32_t* bm,
                          bool check) -> uint64_t {
      for (uint64_t q = from;; q += kRowTile) {
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kRowItems; ++k) {
          const uint64_t i = q + (uint64_t)k * kBlock + tid;
          bool in_row = false;
          uint32_t d = 0;
          if (i < nx) {
            const K key = X[i];
            in_row = (key >> w) == rk;
            d = (uint32_t)(key & fmask);
          }
          mine += in_row ? 1u : 0u;
          if (check) {
            // candidates: a bit already set (a duplicate, or a tuple of Full) costs a read
            bool want = in_row;
            if (want) want = !(((s_fb[d >> 5] | bm[d >> 5]) >> (d & 31u)) & 1u);
            if (want) atomicOr(&bm[d >> 5], 1u << (d & 31u));
          } else {
            or_sorted_runs(bm, in_row, d);  // Full: sorted, distinct, in lane order
          }
        }
        uint32_t got;
        (void)block_excl_scan<uint32_t>(mine, s_wave, got);  // (two barriers)
        const uint64_t avail = nx > q ? min<uint64_t>(nx - q, kRowTile) : 0;
        if (got < avail || q + kRowTile >= nx) return q + got;
      }
    };
    while (p < hi) {
      const K rk = in[p] >> w;
      for (uint32_t x = tid; x < words; x += kBlock) {
        s_cb[x] = 0u;
        s_fb[x] = 0u;
      }
      __syncthreads();
      // Full's keys of this row first: a row not right after a cursor's is found by a wave
      // search (the keys in between belong to rows without candidates here)
      const bool seek_a = pa < FA && (runA[pa] >> w) < rk;
      const bool seek_b = pb < FB && (runB[pb] >> w) < rk;
      if (seek_a || seek_b) {
        if (wid == 0 && seek_a) {
          const uint64_t v = row_search(pa, FA, [&](uint64_t i) { return (runA[i] >> w) < rk; });
          if (lane_id() == 0) s_at[1] = v;
        } else if (wid == 1 && seek_b) {
          const uint64_t v = row_search(pb, FB, [&](uint64_t i) { return (runB[i] >> w) < rk; });
          if (lane_id() == 0) s_at[2] = v;
        }
        __syncthreads();
        if (seek_a) pa = s_at[1];
        if (seek_b) pb = s_at[2];
      }
      pa = stream_row(runA, FA, pa, rk, s_fb, false);
      pb = stream_row(runB, FB, pb, rk, s_fb, false);
      // then the candidates: only bits in neither bitmap are set
      const uint64_t row_end = stream_row(in, n, p, rk, s_cb, true);
      // new bits: candidates not in Full, numbered in bit order (thread t takes wpt
      // consecutive words, so the scan of the per-thread counts is in word order)
      const uint32_t wpt = words >= kBlock ? words / kBlock : 1u;
      uint32_t cnt = 0;
      for (uint32_t q = 0; q < wpt; ++q) {
        const uint32_t x = tid * wpt + q;
        if (x < words) {
          const uint32_t nw = s_cb[x] & ~s_fb[x];
          s_cb[x] = nw;
          cnt += (uint32_t)__popc(nw);
        }
      }
      uint32_t total;
      uint32_t before = block_excl_scan<uint32_t>(cnt, s_wave, total);
      for (uint32_t q = 0; q < wpt; ++q) {
        const uint32_t x = tid * wpt + q;
        if (x < words) {
          s_pre[x] = before;
          before += (uint32_t)__popc(s_cb[x]);
        }
      }
      __syncthreads();
      const K rlo = rk << w;
      for (uint32_t idx = tid; idx < total; idx += kBlock) {
        // the last word whose prefix is <= idx (equal prefixes belong to empty words before
        // the one holding survivor idx)
        uint32_t a = 0, len = words;
        while (len > 0) {
          const uint32_t half = len >> 1;
          if (s_pre[a + half] <= idx) {
            a += half + 1;
            len -= half + 1;
          } else {
            len = half;
          }
        }
        const uint32_t x = a - 1;
        const uint32_t bit = nth_set_bit(s_cb[x], idx - s_pre[x]);
        tmp[out0 + running + idx] = rlo | (K)(x * 32u + bit);
      }
      running += total;
      p = row_end;
      __syncthreads();
    }
  }
  if (tid == 0) {
    b.bcnt[blockIdx.x] = running;
    b.bstart[blockIdx.x] = out0;
  }
}

// Where the merge of iteration j puts Full, and record j: the delta goes into B (the other B
// buffer), or, when B would outgrow A / kFoldRatio, B folds into A (the other A buffer) and
// the delta alone becomes B.  With an empty delta nothing is merged and both runs stay
// where they are.  (One thread, after the delta of N tuples is in place; F = |Full| before.
// |Full| for the route gates is updated by the merge.)
template <typename K>
__device__ __forceinline__ void record_iteration(Ctrl* ctrl, const Bufs<K>& b, uint32_t j, uint64_t N,
                                                 uint64_t F) {
  const IterRec rp = b.rec[j - 1];
  const uint64_t fb = rp.F - rp.FA;
  const bool fold = N > 0 && fb > 0 && (fb + N) * kFoldRatio > rp.FA;
  IterRec& r = b.rec[j];
  r.N = N;
  r.F = F + N;
  r.FA = fold ? F : rp.FA;
  r.a = fold ? (rp.a ^ 1u) : rp.a;
  r.b = N > 0 ? (rp.b ^ 1u) : rp.b;
  r.fold = fold ? 1u : 0u;
  ctrl->iter = j;
  if (N == 0) ctrl->done = 1;
  else if (ctrl->max_iter != 0 && j >= ctrl->max_iter) ctrl->limit_hit = 1;
}

template <typename K, int ITEMS>
__device__ __forceinline__ void compact_gather(Ctrl* ctrl, int mode, const uint64_t* n_ptr, const K* __restrict__ tmp,
                                               Bufs<K> b, uint32_t j, uint32_t side, uint64_t* s_pre,
                                               uint64_t* s_wave) {
  constexpr uint32_t T = kBlock * ITEMS;  // the tile of the local pass it follows
  const bool filt = (mode & kModeFilter) != 0;
  if (block_stop((!filt && halted(ctrl)) ||
                 gated_out(ctrl, (mode & kModeGateRow) ? 1 : ((mode & kModeGateSort) ? 2 : 0), kRowMin,
                           kRowFullPerCand)))
    return;
  j = iter_cur(ctrl, j);
  // the sort before this compaction is over: a later sort that skips the one-block path
  // must not find its flag (nothing else in this launch reads it)
  // (and the long-row queue of a segmented sort is consumed)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->small_sorted = 0;
    ctrl->seg_long = 0;
  }
  const uint64_t n = *n_ptr;
  const uint64_t N = block_prefix(b.bcnt, gridDim.x, s_pre, s_wave);
  uint64_t lo, hi;
  block_range(n, compact_span(n, T, gridDim.x), lo, hi);
  K* out1 = nullptr;
  K* out2 = nullptr;
  K* out3 = nullptr;
  uint32_t ovf = 0;
  uint64_t F = 0;
  if (mode & kModeIter) {
    F = b.rec[j - 1].F;  // |A| + |B| of iteration j - 1
    out1 = b.delta[j & 1u];
    if (F + N > ctrl->full_cap) ovf |= 2u;
    if (N > ctrl->cand_cap) ovf |= 4u;
  } else if (mode & kModeEdges) {
    out1 = b.E;
    if (mode & kModeSeed) {
      out2 = b.full[0];
      out3 = b.delta[0];
      if (N > ctrl->full_cap || N > ctrl->cand_cap) ovf |= 2u;
    }
  } else if (mode & kModeSeed) {
    out1 = b.full[0];
    out2 = b.delta[0];
    if (N > ctrl->full_cap || N > ctrl->cand_cap) ovf |= 2u;
  } else if (mode & kModeDedup) {
    out1 = b.cand[side];  // the input buffer: the local pass has read all of it
  } else {
    out1 = b.full[side ^ 1u];
  }
  if (ovf) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (mode & kModeIter) b.rec[j].N = N;
      atomicOr(&ctrl->overflow, ovf);
    }
    return;
  }
  const uint64_t cnt = b.bcnt[blockIdx.x];
  const uint64_t pre = s_pre[blockIdx.x];
  for (uint64_t t = threadIdx.x; t < cnt; t += kBlock) {
    const K v = tmp[lo + t];
    out1[pre + t] = v;
    if (out2) out2[pre + t] = v;
    if (out3) out3[pre + t] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (mode & kModeIter) {
      record_iteration<K>(ctrl, b, j, N, F);
    } else if (mode & (kModeEdges | kModeSeed)) {
      if (mode & kModeEdges) ctrl->m_unique = N;
      if (mode & kModeSeed) {
        IterRec& r = b.rec[0];
        r.N = N;
        r.F = N;
        r.FA = N;  // the seed is run A (Full[0]); run B starts empty
        r.a = 0;
        r.b = 0;
        r.fold = 0;
        ctrl->iter = 0;
        ctrl->full_n = N;
        if (N == 0) ctrl->done = 1;
      }
    } else if (mode & kModeDedup) {
      ctrl->dedup_n = N;
    } else {
      ctrl->filtered = N;
    }
  }
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_compact_gather(Ctrl* ctrl, int mode, const uint64_t* n_ptr,
                                                           const K* __restrict__ tmp, Bufs<K> b,
                                                           uint32_t j, uint32_t side) {
  __shared__ uint64_t s_pre[kScanBlocksMax];
  __shared__ uint64_t s_wave[kWavesPerBlock];
  compact_gather<K, ITEMS>(ctrl, mode, n_ptr, tmp, b, j, side, s_pre, s_wave);
}

// The row pass's gather: the survivors of every row-pass block (kRowBlocks of them), in block
// order, to delta[j & 1], and record j as the compaction's gather does.  Each block adds up
// all kRowBlocks totals and copies blocks b, b + G, ...
template <typename K>
__global__ __launch_bounds__(kBlock) void k_row_gather(int gate, Ctrl* ctrl, const K* __restrict__ tmp, Bufs<K> b,
                                                       uint32_t j) {
  __shared__ uint64_t s_pre[kRowBlocks];
  __shared__ uint64_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl) || gated_out(ctrl, gate, kRowMin, kRowFullPerCand))) return;
  j = iter_cur(ctrl, j);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->small_sorted = 0;
    ctrl->seg_long = 0;
  }
  static_assert(kRowBlocks % kBlock == 0, "");
  const uint64_t N = block_prefix<kRowBlocks / kBlock>(b.bcnt, (int)kRowBlocks, s_pre, s_wave);
  const uint64_t F = b.rec[j - 1].F;
  uint32_t ovf = 0;
  if (F + N > ctrl->full_cap) ovf |= 2u;
  if (N > ctrl->cand_cap) ovf |= 4u;
  if (ovf) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      b.rec[j].N = N;
      atomicOr(&ctrl->overflow, ovf);
    }
    return;
  }
  K* __restrict__ out = b.delta[j & 1u];
  for (uint32_t r = blockIdx.x; r < kRowBlocks; r += gridDim.x) {
    const uint64_t cnt = b.bcnt[r];
    const uint64_t src = b.bstart[r];
    const uint64_t dst = s_pre[r];
    for (uint64_t t = threadIdx.x; t < cnt; t += kBlock) out[dst + t] = tmp[src + t];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) record_iteration<K>(ctrl, b, j, N, F);
}

// ---------------------------------------------------------------------------
// Disjoint merge (Section IV-C).  The inputs are disjoint by construction, so the output
// has exactly the sum of their sizes and each tile's slice of both inputs is fixed by a
// merge-path diagonal search: no atomics, no cleanup pass.  Tiles that take keys from one
// input only are straight copies.  Full is two runs (see IterRec): iteration j merges its
// delta into run B or, on a fold, B into A, each into the other buffer of a ping-pong
// pair (Section V-C).
// ---------------------------------------------------------------------------
// Number of A keys among the first `diag` keys of merge(A, B), found by the whole wave.
template <typename K>
__device__ __forceinline__ uint64_t wave_merge_path(const K* A, uint64_t na, const K* B, uint64_t nb,
                                                    uint64_t diag) {
  const uint64_t lo = diag > nb ? diag - nb : 0;
  const uint64_t hi = diag < na ? diag : na;
  return wave_partition(lo, hi, [&](uint64_t i) { return A[i] < B[diag - 1 - i]; });
}

// Tiles of merge(A, B): block `bid` of `nblocks` takes a contiguous range of tiles; output
// position p gets key v through put(p, v) (a store into O, or the split unpack).  Only the
// range's first split is searched over the whole merge path; every later split is
// searched within one tile's worth of A past the previous split, which keeps the
// searches' scattered reads to a small fraction of the data moved.  The loop runs one
// tile ahead: while a tile merges in LDS, wave 0 searches the next tile's end split, and
// the next tile's keys are loaded into registers while this tile's output is written, so
// a tile costs one exposed round of loads instead of three.  s_i: 4 words.
template <typename K, int ITEMS, typename Put>
__device__ __forceinline__ void merge_tiles_to(const K* __restrict__ A, uint64_t na, const K* __restrict__ B,
                                               uint64_t nb, Put put, K* s_in, K* s_out, uint64_t* s_i,
                                               uint32_t bid, uint32_t nblocks) {
  constexpr uint32_t T = kBlock * ITEMS;
  const uint64_t total = na + nb;
  const uint64_t ntiles = (total + T - 1) / T;
  const uint64_t tpb = (ntiles + nblocks - 1) / nblocks;
  const uint64_t t_begin = (uint64_t)bid * tpb;
  const uint64_t t_end = min(t_begin + tpb, ntiles);
  if (t_begin >= t_end) return;
  const int wid = threadIdx.x / kWave;
  // the first tile's two splits, searched at once by two waves
  if (wid == 0) {
    const uint64_t i = wave_merge_path(A, na, B, nb, t_begin * T);
    if (lane_id() == 0) s_i[0] = i;
  } else if (wid == 1) {
    const uint64_t i = wave_merge_path(A, na, B, nb, min((t_begin + 1) * T, total));
    if (lane_id() == 0) s_i[1] = i;
  }
  __syncthreads();
  uint64_t i0 = s_i[0], i1 = s_i[1];
  // keys of output positions [o0, o1): A[a0, a1) then B from o0 - a0, thread-strided
  K reg[ITEMS];
  auto fetch = [&](uint64_t o0, uint64_t o1, uint64_t a0, uint64_t a1) {
    const uint32_t ca = (uint32_t)(a1 - a0), cn = (uint32_t)(o1 - o0);
    const uint64_t b0 = o0 - a0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t t = (uint32_t)k * kBlock + threadIdx.x;
      reg[k] = t < cn ? (t < ca ? A[a0 + t] : B[b0 + (t - ca)]) : K(0);
    }
  };
  fetch(t_begin * T, min((t_begin + 1) * T, total), i0, i1);
  for (uint64_t tile = t_begin; tile < t_end; ++tile) {
    const uint64_t o0 = tile * T;
    const uint64_t o1 = min(o0 + T, total);
    const bool more = tile + 1 < t_end;
    uint64_t* const next = s_i + 2 + ((tile - t_begin) & 1);  // alternates: no reader overlap
    if (more && wid == 0) {
      // the next tile's end split: A keys among the first n1 outputs lie in
      // [max(i1, n1 - nb), min(i1 + (n1 - o1), na)]
      const uint64_t n1 = min(o1 + T, total);
      const uint64_t lo = max(i1, n1 > nb ? n1 - nb : 0);
      const uint64_t hi = min(i1 + (n1 - o1), na);
      // (32-bit keys: an 8-probe first round halves the lines the search touches; its
      // extra round is hidden behind the merge.  64-bit keys measured no gain from it.)
      const auto pred = [&](uint64_t i) { return A[i] < B[n1 - 1 - i]; };
      uint64_t i2;
      if constexpr (sizeof(K) == 4) i2 = wave_partition_fan<8>(lo, hi, pred);
      else i2 = wave_partition(lo, hi, pred);
      if (lane_id() == 0) *next = i2;
    }
    const uint32_t ca = (uint32_t)(i1 - i0), cn = (uint32_t)(o1 - o0), cb = cn - ca;
    if (ca == 0 || cb == 0) {
      // keys of one input only: already in order
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t t = (uint32_t)k * kBlock + threadIdx.x;
        if (t < cn) put(o0 + t, reg[k]);
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t t = (uint32_t)k * kBlock + threadIdx.x;
        if (t < cn) s_in[t] = reg[k];
      }
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
    }
    // next tile's keys in flight while this one's output goes out
    uint64_t i2 = 0;
    if (more) {
      i2 = *next;
      fetch(o1, min(o1 + T, total), i1, i2);
    }
    if (ca != 0 && cb != 0) {
      for (uint32_t t = threadIdx.x; t < cn; t += kBlock) put(o0 + t, s_out[t]);
      __syncthreads();  // s_out is rewritten by the next tile
    }
    i0 = i1;
    i1 = i2;
  }
}

template <typename K, int ITEMS>
__device__ __forceinline__ void merge_tiles(const K* __restrict__ A, uint64_t na, const K* __restrict__ B,
                                            uint64_t nb, K* __restrict__ O, K* s_in, K* s_out,
                                            uint64_t* s_i, uint32_t bid, uint32_t nblocks) {
  merge_tiles_to<K, ITEMS>(A, na, B, nb, [O](uint64_t p, K v) { O[p] = v; }, s_in, s_out, s_i, bid,
                           nblocks);
}

// Iteration j: B' = merge(B, delta^j) into the other B buffer, or on a fold
// A' = merge(A, B) into the other A buffer and B' = delta^j.  The two parts of a fold
// write different buffers and share the grid (one launch per iteration either way).
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_merge(Ctrl* ctrl, Bufs<K> b, uint32_t j) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_in[T];
  __shared__ K s_out[T];
  __shared__ uint64_t s_i[4];
  if (block_stop(halted(ctrl))) return;
  j = iter_cur(ctrl, j);
  const IterRec rp = b.rec[j - 1];
  const IterRec rj = b.rec[j];
  // |Full| for the route gates of the next iteration; set here, not by the gather that
  // records the iteration, whose other blocks read it in their own gate
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->full_n = rj.F;
  const uint64_t fb = rp.F - rp.FA;
  const K* __restrict__ delta = b.delta[j & 1u];
  K* __restrict__ outB = b.fullB[rp.b ^ 1u];
  if (!rj.fold) {
    merge_tiles<K, ITEMS>(b.fullB[rp.b], fb, delta, rj.N, outB, s_in, s_out, s_i, blockIdx.x,
                          gridDim.x);
    return;
  }
  // blocks [0, ga) fold A and B, blocks [ga, grid) copy the delta, in proportion to size
  const uint64_t fold_n = rp.FA + fb;
  uint32_t ga = (uint32_t)((double)gridDim.x * (double)fold_n / (double)(fold_n + rj.N));
  ga = max(1u, min(ga, gridDim.x - 1));
  if (blockIdx.x < ga)
    merge_tiles<K, ITEMS>(b.full[rp.a], rp.FA, b.fullB[rp.b], fb, b.full[rp.a ^ 1u], s_in, s_out, s_i,
                          blockIdx.x, ga);
  else
    merge_tiles<K, ITEMS>(delta, rj.N, delta, 0, outB, s_in, s_out, s_i, blockIdx.x - ga,
                          gridDim.x - ga);
}

// After a tail loop: B' = merge(B, T) into the other B buffer, the side the loop's records
// name (nothing when T is empty).
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_tail_fold(Ctrl* ctrl, Bufs<K> b) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_in[T];
  __shared__ K s_out[T];
  __shared__ uint64_t s_i[4];
  const uint64_t tn = ctrl->tail_n;
  if (block_stop(tn == 0)) return;
  const uint32_t side = ctrl->tail_b;
  const IterRec r = b.rec[ctrl->iter];
  merge_tiles<K, ITEMS>(b.fullB[side], r.F - r.FA - tn, b.tail, tn, b.fullB[side ^ 1u], s_in, s_out, s_i,
                        blockIdx.x, gridDim.x);
}

// O = merge(A, B), sizes from the host (the final union of the two runs).
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_merge_pair(const K* __restrict__ A, uint64_t na,
                                                       const K* __restrict__ B, uint64_t nb,
                                                       K* __restrict__ O) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_in[T];
  __shared__ K s_out[T];
  __shared__ uint64_t s_i[4];
  merge_tiles<K, ITEMS>(A, na, B, nb, O, s_in, s_out, s_i, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Edge index: E is sorted once and never modified (Section IV-A), so the edges of each
// (inst, src) row are contiguous.  U lists the distinct rows, R their starts.  Two
// launches: per-block row-head counts, then every block writes its heads.
// ---------------------------------------------------------------------------
// Dense edge index: Edst, and R[v] = first edge of row v for every row id v <= b.dense
// (R[b.dense] = |E|), each edge filling the rows between its predecessor's row and its own.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_index_dense(Ctrl* ctrl, Bufs<K> b, int w) {
  // R[v] is the first edge whose row is >= v.  Edge i (and the end, i = n) owns the rows
  // after its predecessor's row up to its own, (row(E[i-1]), row(E[i])], and writes i
  // there; these intervals tile [0, dense], so every entry is written once and the work
  // is O(n + dense).  Gaps longer than kGapSerial rows (empty id ranges, e.g. the ids an
  // instance of a batch does not use) are filled by the whole block.
  constexpr uint64_t kGapSerial = 32;
  __shared__ uint32_t s_n;
  __shared__ uint64_t s_from[kBlock], s_to[kBlock];
  __shared__ uint32_t s_val[kBlock];
  if (block_stop(halted(ctrl))) return;
  const uint64_t n = ctrl->m_unique;
  const K* __restrict__ E = b.E;
  const K mask = field_mask<K>(w);
  const uint64_t dense = b.dense;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base <= n; base += (uint64_t)gridDim.x * kBlock) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const uint64_t i = base + threadIdx.x;
    if (i <= n) {
      if (i < n) b.Edst[i] = (uint32_t)(E[i] & mask);
      const uint64_t to = i < n ? (uint64_t)(E[i] >> w) : dense;
      const uint64_t from = i > 0 ? (uint64_t)(E[i - 1] >> w) + 1 : 0;
      if (from <= to) {
        if (to - from < kGapSerial) {
          for (uint64_t v = from; v <= to; ++v) b.R[v] = (uint32_t)i;
        } else {
          const uint32_t q = atomicAdd(&s_n, 1u);
          s_from[q] = from;
          s_to[q] = to;
          s_val[q] = (uint32_t)i;
        }
      }
    }
    __syncthreads();
    const uint32_t ng = s_n;
    for (uint32_t g = 0; g < ng; ++g) {
      const uint64_t to = s_to[g];
      const uint32_t val = s_val[g];
      for (uint64_t v = s_from[g] + threadIdx.x; v <= to; v += kBlock) b.R[v] = val;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->nu = b.dense;
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_index_count(Ctrl* ctrl, Bufs<K> b, int w) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint64_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl))) return;
  const uint64_t n = ctrl->m_unique;
  const K* __restrict__ E = b.E;
  const K mask = field_mask<K>(w);
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  uint64_t cnt = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const K e = E[i];
    b.Edst[i] = (uint32_t)(e & mask);
    if (i == 0 || (e >> w) != (E[i - 1] >> w)) ++cnt;
  }
  uint64_t total;
  block_excl_scan<uint64_t>(cnt, s_wave, total);
  if (threadIdx.x == 0) b.bcnt[blockIdx.x] = total;
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_index_write(Ctrl* ctrl, Bufs<K> b, int w) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ uint64_t s_pre[kScanBlocksMax];
  __shared__ uint64_t s_wave[kWavesPerBlock];
  if (block_stop(halted(ctrl))) return;
  const uint64_t n = ctrl->m_unique;
  const K* __restrict__ E = b.E;
  const uint64_t nu = block_prefix(b.bcnt, gridDim.x, s_pre, s_wave);
  uint64_t lo, hi;
  block_range(n, T, lo, hi);
  uint64_t run = s_pre[blockIdx.x];
  for (uint64_t base = lo; base < hi; base += kBlock) {
    const uint64_t i = base + threadIdx.x;
    bool head = false;
    K e = 0;
    if (i < hi) {
      e = E[i];
      head = (i == 0 || (e >> w) != (E[i - 1] >> w));
    }
    uint64_t total;
    const uint64_t ex = block_excl_scan<uint64_t>(head ? 1ull : 0ull, s_wave, total);
    if (head) {
      b.U[run + ex] = (uint32_t)(e >> w);
      b.R[run + ex] = (uint32_t)i;
    }
    run += total;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->nu = nu;
    b.R[nu] = (uint32_t)n;
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

// The result held as two disjoint sorted runs (Full's A and B): merge them while
// splitting the keys into src and dst arrays.
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_unpack_merge(const K* __restrict__ A, uint64_t na,
                                                         const K* __restrict__ B, uint64_t nb, int w,
                                                         uint32_t* __restrict__ src,
                                                         uint32_t* __restrict__ dst) {
  constexpr uint32_t T = kBlock * ITEMS;
  __shared__ K s_in[T];
  __shared__ K s_out[T];
  __shared__ uint64_t s_i[4];
  const K mask = field_mask<K>(w);
  merge_tiles_to<K, ITEMS>(
      A, na, B, nb,
      [=](uint64_t p, K v) {
        src[p] = (uint32_t)((v >> w) & mask);
        dst[p] = (uint32_t)(v & mask);
      },
      s_in, s_out, s_i, blockIdx.x, gridDim.x);
}

// Per-instance result offsets: out[i] = first key of instance i, out[num] = n.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_offsets(const K* __restrict__ keys, uint64_t n, int shift,
                                                    uint32_t num, uint64_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i <= num;
       i += (uint64_t)gridDim.x * kBlock)
    out[i] = (i == num) ? n : lower_bound<K>(keys, n, (K)i << shift);
}

// The same over two disjoint runs: a key's position in their union is the number of keys
// below it in both.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_offsets2(const K* __restrict__ A, uint64_t na,
                                                     const K* __restrict__ B, uint64_t nb, int shift,
                                                     uint32_t num, uint64_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i <= num;
       i += (uint64_t)gridDim.x * kBlock)
    out[i] = (i == num) ? na + nb
                        : lower_bound<K>(A, na, (K)i << shift) + lower_bound<K>(B, nb, (K)i << shift);
}

// The control block written from a kernel argument (captured when the launch is enqueued, so
// no host staging buffer has to outlive the call that queues it).
__global__ void k_ctrl_set(Ctrl* ctrl, Ctrl v) {
  if (threadIdx.x == 0) *ctrl = v;
}

__global__ void k_resume(Ctrl* ctrl, uint64_t cand_cap, uint64_t full_cap, uint32_t clear_hook) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctrl->cand_cap = cand_cap;
    ctrl->full_cap = full_cap;
    ctrl->overflow = 0;
    ctrl->small_sorted = 0;
    ctrl->seg_long = 0;
    if (clear_hook) ctrl->force_overflow_at = 0;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// Launch with optional start / stop events stamped by the dispatch itself (timing that
// agrees with a kernel trace; no marker packets between kernels).
#define WG_LAUNCH(kernel, grid, start, stop, s, ...)                                            \
  do {                                                                                           \
    if ((start) || (stop))                                                                       \
      hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, start, stop, 0, __VA_ARGS__); \
    else                                                                                         \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__);                   \
  } while (0)

// The same for the one-block kernels of kSmallSortThreads threads.
#define WG_LAUNCH_WIDE(kernel, grid, start, stop, s, ...)                                        \
  do {                                                                                           \
    if ((start) || (stop))                                                                       \
      hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kSmallSortThreads), 0, s, start, stop, 0,    \
                            __VA_ARGS__);                                                        \
    else                                                                                         \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kSmallSortThreads), 0, s, __VA_ARGS__);        \
  } while (0)

static inline int stream_blocks(const Grid& g, uint64_t n) {
  const uint64_t need = (n + kBlock - 1) / kBlock;
  return (int)(need < (uint64_t)g.stream ? (need ? need : 1) : (uint64_t)g.stream);
}

void launch_max_id(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint32_t* src,
                   const uint32_t* dst, uint64_t m) {
  hipLaunchKernelGGL(k_max_id, dim3(stream_blocks(g, m)), dim3(kBlock), 0, s, ctrl, src, dst, m);
}

void launch_check_offsets(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* offsets,
                          uint32_t num, uint64_t m) {
  hipLaunchKernelGGL(k_check_offsets, dim3(stream_blocks(g, num)), dim3(kBlock), 0, s, ctrl, offsets,
                     num, m);
}

template <typename K>
void launch_pack_batch(hipStream_t s, const Grid& g, const uint32_t* src, const uint32_t* dst,
                       uint64_t m, int w, const uint64_t* offsets, uint32_t num, K* keys, Ev ev) {
  WG_LAUNCH(k_pack_batch<K>, stream_blocks(g, m), ev.start, ev.stop, s, src, dst, m, w, offsets, num,
            keys);
}

template <typename K>
void launch_offsets(hipStream_t s, const Grid& g, const K* keys, uint64_t n, const K* keys2, uint64_t n2,
                    int shift, uint32_t num, uint64_t* out) {
  if (n2 == 0)
    hipLaunchKernelGGL(k_offsets<K>, dim3(stream_blocks(g, (uint64_t)num + 1)), dim3(kBlock), 0, s, keys, n,
                       shift, num, out);
  else
    hipLaunchKernelGGL(k_offsets2<K>, dim3(stream_blocks(g, (uint64_t)num + 1)), dim3(kBlock), 0, s, keys,
                       n, keys2, n2, shift, num, out);
}

template <typename K>
void launch_pack(hipStream_t s, const Grid& g, const uint32_t* src, const uint32_t* dst,
                 uint64_t m, int w, K* keys, Ev ev) {
  WG_LAUNCH(k_pack<K>, stream_blocks(g, m), ev.start, ev.stop, s, src, dst, m, w, keys);
}

template <typename K>
void launch_join_count(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w,
                       uint32_t j, Ev ev) {
  if ((kind == kJoinTC || kind == kJoinTri) && b.hrows)
    WG_LAUNCH((k_join_count<K, kJoinTC, kJoinItems, true>), g.scan, ev.start, ev.stop, s, ctrl, b, w, j);
  else if (kind == kJoinTC)
    WG_LAUNCH((k_join_count<K, kJoinTC, kJoinItems>), g.scan, ev.start, ev.stop, s, ctrl, b, w, j);
  else if (kind == kJoinSG)
    WG_LAUNCH((k_join_count<K, kJoinSG, kJoinItems>), g.scan, ev.start, ev.stop, s, ctrl, b, w, j);
  else if (kind == kJoinTri)  // counts as the TC join
    WG_LAUNCH((k_join_count<K, kJoinTC, kJoinItems>), g.scan, ev.start, ev.stop, s, ctrl, b, w, j);
  else
    WG_LAUNCH((k_join_count<K, kJoinSGBase, kJoinItems>), g.scan, ev.start, ev.stop, s, ctrl, b, w, j);
}

template <typename K>
void launch_hash_rows(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, Ev ev) {
  const uint64_t slots = (uint64_t)b.hrows + 1 + (b.hpairs ? (uint64_t)b.hpairs + 1 : 0);
  const hipEvent_t none = nullptr;
  WG_LAUNCH(k_fill_u64, g.stream, ev.start, none, s, b.htab, slots, kHashVacant);
  WG_LAUNCH((k_hash_rows_build<K>), g.stream, none, b.hpairs ? none : ev.stop, s, ctrl, b);
  if (b.hpairs) WG_LAUNCH((k_hash_pairs_build<K>), g.stream, none, ev.stop, s, ctrl, b);
}

template <typename K>
void launch_hash_build(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w, uint64_t slots,
                       Ev ev) {
  hipEvent_t none = nullptr;
  WG_LAUNCH(k_fill_u64, stream_blocks(g, slots), ev.start, none, s, b.htab, slots, kHashEmpty);
  WG_LAUNCH(k_hash_build<K>, g.stream, none, ev.stop, s, ctrl, b, w, (uint32_t)(slots - 1));
}

template <typename K>
void launch_join_hash(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w,
                      uint32_t j, uint64_t slots, Ev ev_count, Ev ev_emit) {
  const uint32_t mask = (uint32_t)(slots - 1);
  WG_LAUNCH((k_join_count_hash<K, kJoinTC, kJoinItems>), g.scan, ev_count.start, ev_count.stop, s, ctrl, b, w,
            j, mask);
  if (kind == kJoinTri)
    WG_LAUNCH((k_join_emit_hash<K, kJoinTri, kJoinItems>), g.scan, ev_emit.start, ev_emit.stop, s, ctrl, b, w,
              j, mask);
  else
    WG_LAUNCH((k_join_emit_hash<K, kJoinTC, kJoinItems>), g.scan, ev_emit.start, ev_emit.stop, s, ctrl, b, w,
              j, mask);
}

template <typename K, int ITEMS>
void join_emit_impl(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w, uint32_t j,
                    Ev ev) {
  if (kind == kJoinTC)
    WG_LAUNCH((k_join_emit<K, kJoinTC, ITEMS>), g.stream, ev.start, ev.stop, s, ctrl, b, w, j, g.scan);
  else if (kind == kJoinSG)
    WG_LAUNCH((k_join_emit<K, kJoinSG, ITEMS>), g.stream, ev.start, ev.stop, s, ctrl, b, w, j, g.scan);
  else if (kind == kJoinTri && b.hpairs)
    WG_LAUNCH((k_join_emit<K, kJoinTri, ITEMS, true>), g.stream, ev.start, ev.stop, s, ctrl, b, w, j, g.scan);
  else if (kind == kJoinTri)
    WG_LAUNCH((k_join_emit<K, kJoinTri, ITEMS>), g.stream, ev.start, ev.stop, s, ctrl, b, w, j, g.scan);
  else
    WG_LAUNCH((k_join_emit<K, kJoinSGBase, ITEMS>), g.stream, ev.start, ev.stop, s, ctrl, b, w, j, g.scan);
}

template <typename K>
void launch_join_emit(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w,
                      uint32_t j, Ev ev, bool narrow) {
  if (narrow && kind != kJoinTri && kind != kJoinSGBase)
    join_emit_impl<K, kEmitItemsNarrow>(s, g, kind, ctrl, b, w, j, ev);
  else
    join_emit_impl<K, kEmitItems>(s, g, kind, ctrl, b, w, j, ev);
}

template <typename K, int RB, int ITEMS>
void sort_pass_impl(hipStream_t s, Ctrl* ctrl, const uint64_t* n_ptr, int G, const Bufs<K>& b, int p,
                    bool scatter, Ev ev) {
  constexpr uint32_t T = kBlock * ITEMS;
  const K* in = b.cand[p & 1];
  K* out = b.cand[(p + 1) & 1];
  hipEvent_t none = nullptr;
  if (!scatter) {
    WG_LAUNCH((k_radix_count<K, RB, ITEMS>), G, ev.start, none, s, ctrl, n_ptr, in, p * RB, b.rcnt);
    WG_LAUNCH(k_radix_scan, 1 << RB, none, ev.stop, s, ctrl, n_ptr, T, b.rcnt, b.rtot, G);
  } else {
    WG_LAUNCH((k_radix_scatter<K, RB, ITEMS>), G, ev.start, ev.stop, s, ctrl, n_ptr, in, out, p * RB,
              b.rcnt, b.rtot);
  }
}

template <typename K>
void launch_seg_sort(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b, int w,
                     int passes, bool long_rows, Ev ev, int gate) {
  const int G = std::max(1, g.scan / 2);
  K* out = b.cand[passes & 1];
  const hipEvent_t none = nullptr;
  // the long-row queue lives in b.off, free between the emit that fills it per delta tuple
  // and the next iteration's join count (at most n / kSegBitonicMax rows of three words)
  WG_LAUNCH_WIDE((k_seg_sort<K>), G, ev.start, long_rows ? none : ev.stop, s, gate, ctrl, n_ptr, (const K*)b.cand[0],
                 out, w, b.off, long_rows ? 1 : 0);
  if (long_rows)
    WG_LAUNCH_WIDE((k_seg_long<K>), g.scan, none, ev.stop, s, gate, ctrl, (const K*)b.cand[0], out, w,
                   (const uint32_t*)b.off);
}

template <typename K>
void launch_small_sort(hipStream_t s, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b, int passes,
                       bool alone, Ev ev) {
  const uint32_t a = alone ? 1u : 0u;
  if (ev.start || ev.stop)
    hipExtLaunchKernelGGL(k_small_sort<K>, dim3(1), dim3(kSmallSortThreads), 0, s, ev.start, ev.stop, 0, ctrl,
                          n_ptr, (const K*)b.cand[0], b.cand[passes & 1], a);
  else
    hipLaunchKernelGGL(k_small_sort<K>, dim3(1), dim3(kSmallSortThreads), 0, s, ctrl, n_ptr,
                       (const K*)b.cand[0], b.cand[passes & 1], a);
}

template <typename K>
void launch_small_join(hipStream_t s, int kind, Ctrl* ctrl, const Bufs<K>& b, int w, uint32_t j, int passes,
                       Ev ev) {
  K* out = b.cand[passes & 1];
  const dim3 G(1), B(kSmallSortThreads);
  if (kind == kJoinTC) {
    if (ev.start || ev.stop)
      hipExtLaunchKernelGGL((k_small_join<K, kJoinTC>), G, B, 0, s, ev.start, ev.stop, 0, ctrl, b, w, j, out);
    else
      hipLaunchKernelGGL((k_small_join<K, kJoinTC>), G, B, 0, s, ctrl, b, w, j, out);
  } else {
    if (ev.start || ev.stop)
      hipExtLaunchKernelGGL((k_small_join<K, kJoinSG>), G, B, 0, s, ev.start, ev.stop, 0, ctrl, b, w, j, out);
    else
      hipLaunchKernelGGL((k_small_join<K, kJoinSG>), G, B, 0, s, ctrl, b, w, j, out);
  }
}

template <typename K>
void launch_sort_pass(hipStream_t s, Ctrl* ctrl, const uint64_t* n_ptr, const SortCfg& c,
                      const Bufs<K>& b, int pass, bool scatter, Ev ev) {
  constexpr int SMALL = 8;
  constexpr int LARGE = sizeof(K) == 4 ? 16 : 12;
  const bool large = c.items != SMALL;
  const int G = c.blocks;
  switch (c.rb) {
#define WG_SORT_CASE(RB)                                                                 \
    case RB:                                                                             \
      if (large) sort_pass_impl<K, RB, LARGE>(s, ctrl, n_ptr, G, b, pass, scatter, ev);  \
      else sort_pass_impl<K, RB, SMALL>(s, ctrl, n_ptr, G, b, pass, scatter, ev);        \
      break;
    WG_SORT_CASE(8)
    WG_SORT_CASE(9)
    WG_SORT_CASE(10)
    WG_SORT_CASE(11)
#undef WG_SORT_CASE
    default:
      break;
  }
}

template <typename K>
void launch_compact(hipStream_t s, const Grid& g, int mode, Ctrl* ctrl, const uint64_t* n_ptr,
                    const K* in, K* tmp, const Bufs<K>& b, int w, uint32_t j, uint32_t side, Ev ev, bool narrow) {
  hipEvent_t none = nullptr;
  if (narrow) {
    WG_LAUNCH((k_compact_local<K, kDedupItemsNarrow>), g.scan, ev.start, none, s, ctrl, mode, n_ptr, in, tmp,
              b, w, j);
    WG_LAUNCH((k_compact_gather<K, kDedupItemsNarrow>), g.scan, none, ev.stop, s, ctrl, mode, n_ptr, tmp, b,
              j, side);
  } else {
    WG_LAUNCH((k_compact_local<K, kDedupItems>), g.scan, ev.start, none, s, ctrl, mode, n_ptr, in, tmp, b, w,
              j);
    WG_LAUNCH((k_compact_gather<K, kDedupItems>), g.scan, none, ev.stop, s, ctrl, mode, n_ptr, tmp, b, j,
              side);
  }
}

template <typename K>
void launch_row_diff(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b, int w,
                     uint32_t j, Ev ev, int gate) {
  (void)g;
  WG_LAUNCH((k_row_diff<K>), kRowBlocks, ev.start, ev.stop, s, gate, ctrl, n_ptr, (const K*)b.cand[0], b.cand[1], b,
            w, j);
}

template <typename K>
void launch_row_gather(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b,
                       uint32_t j, Ev ev, int gate) {
  (void)n_ptr;
  WG_LAUNCH((k_row_gather<K>), g.scan, ev.start, ev.stop, s, gate, ctrl, (const K*)b.cand[1], b, j);
}

template <typename K>
void launch_merge(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, uint32_t j, Ev ev) {
  WG_LAUNCH((k_merge<K, kMergeItems>), g.stream, ev.start, ev.stop, s, ctrl, b, j);
}

template <typename K>
void launch_tail_loop(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w, uint32_t jmax,
                      Ev ev, Ev ev_fold) {
  if (kind == kJoinTC)
    WG_LAUNCH_WIDE((k_tail_loop<K, kJoinTC>), 1, ev.start, ev.stop, s, ctrl, b, w, jmax);
  else
    WG_LAUNCH_WIDE((k_tail_loop<K, kJoinSG>), 1, ev.start, ev.stop, s, ctrl, b, w, jmax);
  WG_LAUNCH((k_tail_fold<K, kMergeItems>), g.stream, ev_fold.start, ev_fold.stop, s, ctrl, b);
}

template <typename K>
void launch_merge_pair(hipStream_t s, const Grid& g, const K* A, uint64_t na, const K* B, uint64_t nb,
                       K* O, Ev ev) {
  WG_LAUNCH((k_merge_pair<K, kMergeItems>), stream_blocks(g, (na + nb + 7) / 8), ev.start, ev.stop, s, A,
            na, B, nb, O);
}

template <typename K>
void launch_edge_index(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w, Ev ev) {
  if (b.dense) {
    WG_LAUNCH(k_index_dense<K>, g.stream, ev.start, ev.stop, s, ctrl, b, w);
    return;
  }
  hipEvent_t none = nullptr;
  WG_LAUNCH((k_index_count<K, kIndexItems>), g.scan, ev.start, none, s, ctrl, b, w);
  WG_LAUNCH((k_index_write<K, kIndexItems>), g.scan, none, ev.stop, s, ctrl, b, w);
}

template <typename K>
void launch_unpack(hipStream_t s, const Grid& g, const K* keys, uint64_t n, const K* keys2, uint64_t n2, int w,
                   uint32_t* src, uint32_t* dst) {
  if (n2 == 0) {
    hipLaunchKernelGGL(k_unpack<K>, dim3(stream_blocks(g, n)), dim3(kBlock), 0, s, keys, n, w, src, dst);
    return;
  }
  hipLaunchKernelGGL((k_unpack_merge<K, kMergeItems>), dim3(stream_blocks(g, (n + n2 + 7) / 8)), dim3(kBlock), 0,
                     s, keys, n, keys2, n2, w, src, dst);
}

void launch_ctrl_set(hipStream_t s, Ctrl* ctrl, const Ctrl& v) {
  hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(kWave), 0, s, ctrl, v);
}

void launch_resume(hipStream_t s, Ctrl* ctrl, uint64_t cand_cap, uint64_t full_cap, uint32_t clear_hook) {
  hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, ctrl, cand_cap, full_cap, clear_hook);
}

#define WG_INSTANTIATE(K)                                                                          \
  template void launch_pack<K>(hipStream_t, const Grid&, const uint32_t*, const uint32_t*,       \
                               uint64_t, int, K*, Ev);                                            \
  template void launch_pack_batch<K>(hipStream_t, const Grid&, const uint32_t*, const uint32_t*, \
                                     uint64_t, int, const uint64_t*, uint32_t, K*, Ev);           \
  template void launch_offsets<K>(hipStream_t, const Grid&, const K*, uint64_t, const K*, uint64_t, int, \
                                  uint32_t, uint64_t*);                                            \
  template void launch_join_count<K>(hipStream_t, const Grid&, int, Ctrl*, const Bufs<K>&, int,   \
                                     uint32_t, Ev);                                                \
  template void launch_join_emit<K>(hipStream_t, const Grid&, int, Ctrl*, const Bufs<K>&, int,    \
                                    uint32_t, Ev, bool);                                           \
  template void launch_small_sort<K>(hipStream_t, Ctrl*, const uint64_t*, const Bufs<K>&, int, bool, Ev); \
  template void launch_small_join<K>(hipStream_t, int, Ctrl*, const Bufs<K>&, int, uint32_t, int, Ev); \
  template void launch_seg_sort<K>(hipStream_t, const Grid&, Ctrl*, const uint64_t*, const Bufs<K>&, int, int, bool, \
                                   Ev, int);                                                       \
  template void launch_sort_pass<K>(hipStream_t, Ctrl*, const uint64_t*, const SortCfg&,         \
                                    const Bufs<K>&, int, bool, Ev);                                \
  template void launch_compact<K>(hipStream_t, const Grid&, int, Ctrl*, const uint64_t*, const K*, \
                                  K*, const Bufs<K>&, int, uint32_t, uint32_t, Ev, bool);          \
  template void launch_merge<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&, uint32_t, Ev);   \
  template void launch_tail_loop<K>(hipStream_t, const Grid&, int, Ctrl*, const Bufs<K>&, int, uint32_t, Ev, Ev); \
  template void launch_row_diff<K>(hipStream_t, const Grid&, Ctrl*, const uint64_t*, const Bufs<K>&, int, \
                                   uint32_t, Ev, int);                                             \
  template void launch_row_gather<K>(hipStream_t, const Grid&, Ctrl*, const uint64_t*, const Bufs<K>&,  \
                                     uint32_t, Ev, int);                                           \
  template void launch_hash_build<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&, int, uint64_t, Ev); \
  template void launch_hash_rows<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&, Ev);             \
  template void launch_join_hash<K>(hipStream_t, const Grid&, int, Ctrl*, const Bufs<K>&, int, uint32_t, \
                                    uint64_t, Ev, Ev);                                             \
  template void launch_merge_pair<K>(hipStream_t, const Grid&, const K*, uint64_t, const K*,     \
                                     uint64_t, K*, Ev);                                            \
  template void launch_edge_index<K>(hipStream_t, const Grid&, Ctrl*, const Bufs<K>&, int, Ev);   \
  template void launch_unpack<K>(hipStream_t, const Grid&, const K*, uint64_t, const K*, uint64_t, int, \
                                 uint32_t*, uint32_t*);

WG_INSTANTIATE(uint32_t)
WG_INSTANTIATE(uint64_t)

}  // namespace wg

// ---------------------------------------------------------------------------
// wg_sort_keys_noalloc: the LSD sort on caller arrays with no allocation at all.  Its
// scratch -- the control block the passes read their size from, the per-block digit
// counts of one pass and the digit totals -- is the file-scope array below: one copy per
// device, held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, resolved once per device with that device current.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoAllocDigitBits = 8;
constexpr int kNoAllocDigits = 1 << kNoAllocDigitBits;
constexpr int kNoAllocBlocks = 1024;  // count and scatter blocks (at most)
constexpr size_t kNoAllocCtrlBytes = 256;
constexpr size_t kNoAllocCountBytes = sizeof(uint32_t) * kNoAllocDigits * kNoAllocBlocks;
constexpr size_t kNoAllocTotalBytes = sizeof(uint32_t) * kNoAllocDigits;
constexpr size_t kNoAllocScratchBytes = kNoAllocCtrlBytes + kNoAllocCountBytes + kNoAllocTotalBytes;
constexpr uint64_t kNoAllocMaxKeys = 0xFFFFFFF0ull;  // output positions are 32-bit
constexpr int kNoAllocMaxDevices = 64;
static_assert(sizeof(wg::Ctrl) <= kNoAllocCtrlBytes, "control block fits its slot");
static_assert(kNoAllocScratchBytes == WG_SORT_NOALLOC_SCRATCH_BYTES, "header states the scratch size");

std::mutex g_noalloc_mu;
void* g_noalloc_scratch[kNoAllocMaxDevices];  // device address of `scratch` per device
int g_noalloc_blocks[kNoAllocMaxDevices];

}  // namespace

static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

template <typename K>
void sort_noalloc(hipStream_t s, uint8_t* base, int G, K* keys, K* tmp, uint64_t n, uint32_t key_bits) {
  using namespace wg;
  Ctrl* ctrl = (Ctrl*)base;
  Bufs<K> b;
  std::memset(&b, 0, sizeof(b));
  b.cand[0] = keys;
  b.cand[1] = tmp;
  b.rcnt = (uint32_t*)(base + kNoAllocCtrlBytes);
  b.rtot = (uint32_t*)(base + kNoAllocCtrlBytes + kNoAllocCountBytes);
  // every field the passes read: the size, no halting flags, no one-block sort
  Ctrl c0;
  std::memset(&c0, 0, sizeof(c0));
  c0.m_in = n;
  launch_ctrl_set(s, ctrl, c0);
  SortCfg c;
  c.rb = kNoAllocDigitBits;
  c.items = sizeof(K) == 4 ? 16 : 8;  // the engine's default tiles
  c.blocks = G;
  const int passes = sort_passes((int)key_bits, c.rb);
  for (int p = 0; p < passes; ++p) {
    launch_sort_pass<K>(s, ctrl, &ctrl->m_in, c, b, p, false, Ev());
    launch_sort_pass<K>(s, ctrl, &ctrl->m_in, c, b, p, true, Ev());
  }
  if (passes & 1) (void)hipMemcpyAsync(keys, tmp, n * sizeof(K), hipMemcpyDeviceToDevice, s);
}

}  // namespace

extern "C" wg_status wg_sort_keys_noalloc(void* d_keys, void* d_tmp, uint64_t n, uint32_t key_bytes,
                                          uint32_t key_bits, void* stream) {
  if (key_bytes != 4 && key_bytes != 8) {
    wg::set_call_error("wg_sort_keys_noalloc: key_bytes must be 4 or 8");
    return WG_ERR_INVALID_ARG;
  }
  if (key_bits == 0 || key_bits > 8 * key_bytes) {
    wg::set_call_error("wg_sort_keys_noalloc: key_bits must be 1..8*key_bytes");
    return WG_ERR_INVALID_ARG;
  }
  if (n > kNoAllocMaxKeys) {
    wg::set_call_error("wg_sort_keys_noalloc: more than 2^32 - 16 keys");
    return WG_ERR_INVALID_ARG;
  }
  if (n > 0 && (!d_keys || !d_tmp)) {
    wg::set_call_error("wg_sort_keys_noalloc: NULL key array with n > 0");
    return WG_ERR_INVALID_ARG;
  }
  wg::set_call_error("");
  if (n <= 1) return WG_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) {
    (void)hipGetLastError();
    wg::set_call_error("wg_sort_keys_noalloc: no usable current device");
    return WG_ERR_DEVICE;
  }
  uint8_t* base = nullptr;
  int G = 0;
  {
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_scratch[dev]) {
      void* p = nullptr;
      const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      int cu = 0;
      if (r != hipSuccess || !p ||
          hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        wg::set_call_error("wg_sort_keys_noalloc: hipGetSymbolAddress of the scratch array failed");
        return WG_ERR_DEVICE;
      }
      g_noalloc_blocks[dev] = std::max(1, std::min(4 * std::max(cu, 1), kNoAllocBlocks));
      g_noalloc_scratch[dev] = p;
    }
    base = (uint8_t*)g_noalloc_scratch[dev];
    G = g_noalloc_blocks[dev];
  }
  hipStream_t s = (hipStream_t)stream;
  if (key_bytes == 4) sort_noalloc<uint32_t>(s, base, G, (uint32_t*)d_keys, (uint32_t*)d_tmp, n, key_bits);
  else sort_noalloc<uint64_t>(s, base, G, (uint64_t*)d_keys, (uint64_t*)d_tmp, n, key_bits);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) {
    wg::set_call_error("wg_sort_keys_noalloc: launch failed");
    return WG_ERR_DEVICE;
  }
  return WG_OK;
}
