// Host-side launchers of the fixpoint kernels (defined in wg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wg_device.h"

namespace wg {

// Query kinds of the join.
enum JoinKind : int { kJoinTC = 0, kJoinSG = 1, kJoinSGBase = 2 };

// dedup_diff output modes (bit flags).
enum DedupMode : int {
  kModeEdges = 1,  // write the deduplicated relation to `outE`, count -> ctrl->m_unique
  kModeSeed = 2,   // write it to Full[0] and delta[0], count -> F, D, |Delta^0|; done if empty
  kModeIter = 4,   // candidates minus Full -> delta[1 - delta_side], iteration bookkeeping
};

// Lookback / last-block state slots (one per kernel kind).
enum LbSlot : int {
  kLbJoin = 0,
  kLbHist = 1,
  kLbPass = 2,
  kLbDedup = 3,
  kLbMerge = 4,
  kLbIndex = 5,
  kLbFilter = 6,
  kLbCount = 7
};

// Tile sizes (keys per tile) of the lookback kernels; status arrays are sized from them.
constexpr int kJoinItems = 8;
constexpr int kEmitItems = 8;
constexpr int kDedupItems = 8;
constexpr int kMergeItems = 8;
constexpr int kIndexItems = 8;
template <typename K> constexpr int pass_items() { return sizeof(K) == 4 ? 16 : 12; }
template <typename K> constexpr uint32_t pass_tile() { return kBlock * pass_items<K>(); }
constexpr uint32_t kJoinTile = kBlock * kJoinItems;
constexpr uint32_t kDedupTile = kBlock * kDedupItems;
constexpr uint32_t kIndexTile = kBlock * kIndexItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxPasses = 8;
// Blocks of the radix count / scatter kernels (one static key range each).
constexpr int kSortBlocksMax = 4096;

struct Grid {
  int persistent;  // blocks of the lookback kernels
  int stream;      // blocks of grid-stride kernels
  int sort;        // blocks of the radix count / scatter kernels (<= kSortBlocksMax)
};

// Per-iteration device arrays of one solve.
template <typename K>
struct Bufs {
  K* cand[2];
  K* full[2];
  K* delta[2];
  K* E;
  uint32_t* U;     // distinct (inst, src) rows of E, ascending
  uint32_t* R;     // row starts, nu + 1 entries
  uint32_t* Edst;  // destination column of E
  uint32_t* rowa;
  uint32_t* rowb;
  uint32_t* off;
  uint64_t* hist;  // per iteration: [2*i] = |Delta^i|, [2*i+1] = candidates of iteration i
  LbState* lb;     // kLbCount entries
  uint64_t* status[kLbCount];
  uint32_t* rcnt;  // radix per-block digit counts / offsets, kRadix x sort blocks
  uint32_t* rtot;  // radix digit totals, kRadix
};

void launch_max_id(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint32_t* src,
                   const uint32_t* dst, uint64_t m);

template <typename K>
void launch_pack(hipStream_t s, const Grid& g, const uint32_t* src, const uint32_t* dst,
                 uint64_t m, int w, K* keys);

template <typename K>
void launch_join_count(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w);

template <typename K>
void launch_join_emit(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w);

// One stable 8-bit LSD pass: count, scan and scatter launches.
template <typename K>
void launch_radix_pass(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr,
                       const K* in, K* out, int pass, const Bufs<K>& b);

template <typename K>
void launch_dedup_diff(hipStream_t s, const Grid& g, int mode, Ctrl* ctrl, const uint64_t* n_ptr,
                       const K* cand, const Bufs<K>& b);

template <typename K>
void launch_merge(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b);

template <typename K>
void launch_edge_index(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w);

template <typename K>
void launch_filter_offdiag(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w);

template <typename K>
void launch_unpack(hipStream_t s, const Grid& g, const K* keys, uint64_t n, int w,
                   uint32_t* src, uint32_t* dst);

void launch_resume(hipStream_t s, Ctrl* ctrl, uint64_t cand_cap, uint64_t full_cap,
                   uint64_t dsz_cap, uint32_t clear_hook);

}  // namespace wg
