// Host-side launchers of the fixpoint kernels (defined in wg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wg_device.h"

namespace wg {

// Query kinds of the join.
// kJoinTri: the TC join of E with itself whose emit phase probes E for each two-path's
// closing edge instead of writing candidates (triangle counting, Section VI).
enum JoinKind : int { kJoinTC = 0, kJoinSG = 1, kJoinSGBase = 2, kJoinTri = 3 };

// Compaction modes of dedup_local / dedup_gather.
enum CompactMode : int {
  kModeEdges = 1,   // sorted candidates -> E (dedup only), count -> m_unique
  kModeSeed = 2,    // sorted candidates -> Full[0] and delta[0] (dedup only), record 0
  kModeIter = 4,    // sorted candidates minus Full[(j-1)&1] -> delta[j&1], record j
  kModeFilter = 8,  // Full[side] without (x, x) -> Full[side^1], count -> filtered
  // unfused variant: sorted candidates in cand[side] -> deduplicated in place, count ->
  // dedup_n; a kModeIter pass over them then takes the set difference alone
  kModeDedup = 16,
  // gates of an iteration enqueued with both routes (see kRowMin): run only on the row route,
  // or only on the sort route
  kModeGateRow = 64,
  kModeGateSort = 128,
};

// Row pass (TC): ids of at most this many bits get a bitmap per row in LDS.
constexpr int kRowBitsMax = 16;
// A TC iteration may be enqueued with both routes -- the row pass, and the segmented sort
// plus compaction -- when the host cannot tell its size yet: the kernels of each route read
// the join's candidate count and return at once unless it picks their route (the row pass
// from kRowMin candidates on).  gate: 0 none, 1 the row route, 2 the sort route.
constexpr uint64_t kRowMin = 1ull << 21;
// ... and while Full has at most this many tuples per candidate: the row pass costs about
// the candidates plus the touched rows of Full, the sort route (LSD passes and compaction)
// about five times the candidates plus the windows of Full, so the rows win up to a Full of
// some four times the candidates (measured on R-MAT 15: its fifth iteration, 27M candidates
// against 44M tuples of Full, runs twice as fast on the rows).
constexpr uint64_t kRowFullPerCand = 4;
// Blocks of the row pass (four times the compaction's grid: rows are streamed with a barrier
// per round, so more and smaller blocks in flight hide more latency and even out the rows;
// measured on R-MAT 15's largest iteration: 1,024 blocks 752 us, 2,048 451 us, 4,096 blocks
// with half the keys per round 399 us).  Its gather sums this many block totals.
constexpr uint32_t kRowBlocks = 4096;

// Tile sizes (items per tile) of the static-range kernels.
constexpr int kJoinItems = 8;
constexpr int kEmitItems = 8;
constexpr int kDedupItems = 8;
// Narrow tiles of the emit and the compaction (half the keys per tile, half the LDS): for
// iterations of up to a few million candidates, where more blocks in flight and shorter
// per-tile chains win over fewer tiles.
constexpr int kEmitItemsNarrow = 4;
constexpr int kDedupItemsNarrow = 4;
constexpr int kMergeItems = 8;
constexpr uint32_t kSmallSortBytes = 32768;  // LDS of the one-block sort (8,192 / 4,096 keys)
constexpr uint32_t kSmallJoinTuples = 1024;   // delta tuples of the one-block join (one per thread)
constexpr int kIndexItems = 8;
constexpr uint32_t kJoinTile = kBlock * kJoinItems;
constexpr uint32_t kIndexTile = kBlock * kIndexItems;
// Radix digit widths the sort is built for, and its grid limit (the per-block digit
// counts of one pass take (1 << digit bits) x blocks entries).
constexpr int kRadixBitsMin = 8;
constexpr int kRadixBitsMax = 11;
constexpr int kRadixMax = 1 << kRadixBitsMax;
constexpr int kRadixBlocksMax = 2048;
inline int sort_passes(int key_bits, int rb) { return (key_bits + rb - 1) / rb; }

// One configuration of the sort: digit bits, keys per thread and tile (8, or the large
// tile: 16 for 32-bit keys, 12 for 64-bit keys), blocks per pass.
struct SortCfg {
  int rb = 8;
  int items = 0;  // 8 = small tile; anything else = the large tile
  int blocks = 1024;
};
// Blocks of the static-range kernels (join count, radix count/scatter, compaction, index).
// Consumers keep the per-block totals of a launch in LDS, so this is bounded.
constexpr int kScanBlocksMax = 1024;

// Optional events stamped at the start of a stage's first kernel and the end of its last.
struct Ev {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

struct Grid {
  int stream;  // blocks of grid-stride kernels (emit, merge, pack, unpack)
  int scan;    // blocks of the static-range kernels (<= kScanBlocksMax)
};

// Device arrays of one engine (pointer bundle passed by value to every kernel).
template <typename K>
struct Bufs {
  K* cand[2];      // join output / radix ping-pong; the free one is compaction scratch
  K* full[2];      // large run A of Full, ping-pong (side in the records)
  K* fullB[2];     // small run B of Full, ping-pong (side in the records)
  K* delta[2];     // delta ping-pong: iteration j reads side (j-1)&1, writes side j&1
  K* E;            // sorted, deduplicated edge keys
  uint32_t* U;     // distinct (inst, src) rows of E, ascending
  uint32_t* R;     // row starts, nu + 1 entries
  uint32_t* Edst;  // destination column of E
  uint32_t* rowa;  // per delta tuple: row of its head (SG)
  uint32_t* rowb;  // per delta tuple: row of its join vertex
  uint32_t* off;   // per delta tuple: first candidate, relative to its block's range
  uint64_t* jtot;  // per join-count block: candidates of its range
  uint64_t* bcnt;  // per compaction block: survivors of its range
  uint64_t* bstart; // per row-pass block: first position of its survivors in the scratch
                    // (kRowBlocks entries; bcnt has as many)
  uint64_t* hits;  // triangle probe: closing edges found per emit block
  uint64_t* htab;  // hash-join variant: open-addressing table of E (power-of-two slots)
  uint32_t* rcnt;  // radix: per-block digit counts, then offsets (digits x blocks)
  uint32_t* rtot;  // radix: digit totals
  K* tail;         // run T of a tail loop, handed to the fold after it (kTailRunBytes)
  IterRec* rec;    // per-iteration sizes
  uint32_t dense;  // > 0: R is a dense index over the row ids [0, dense) (R[v] = first edge
                   // of row v, R[dense] = |E|) and U is unused; 0: rows are U's entries
  uint32_t hrows;  // fair hash variant: row table htab[0, hrows] (slots - 1), 0 = off
  uint32_t hpairs; // ... and E's pair set htab[hrows + 1, hrows + 1 + hpairs], 0 = none
};

void launch_max_id(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint32_t* src,
                   const uint32_t* dst, uint64_t m);

template <typename K>
void launch_pack(hipStream_t s, const Grid& g, const uint32_t* src, const uint32_t* dst,
                 uint64_t m, int w, K* keys, Ev ev = Ev());

// Batches: validate the instance offsets (sets ctrl->bad_input), pack with the instance
// in the top key bits, and find each instance's first key in the sorted result.
void launch_check_offsets(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* offsets,
                          uint32_t num, uint64_t m);
template <typename K>
void launch_pack_batch(hipStream_t s, const Grid& g, const uint32_t* src, const uint32_t* dst,
                       uint64_t m, int w, const uint64_t* offsets, uint32_t num, K* keys,
                       Ev ev = Ev());
// (of the union of the sorted runs keys[0, n) and keys2[0, n2); n2 may be 0)
template <typename K>
void launch_offsets(hipStream_t s, const Grid& g, const K* keys, uint64_t n, const K* keys2, uint64_t n2,
                    int shift, uint32_t num, uint64_t* out);

// Join of iteration j (kind kJoinSGBase: the base rule, j = 0): count, then emit.
template <typename K>
void launch_join_count(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w,
                       uint32_t j, Ev ev = Ev());
template <typename K>
void launch_join_emit(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w,
                      uint32_t j, Ev ev = Ev(), bool narrow = false);

// Hash-join variant (TC and triangle joins): build the table of E (`slots` a power of
// two), then the count and emit phases of iteration j through it.
template <typename K>
void launch_hash_build(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w, uint64_t slots,
                       Ev ev = Ev());
// Fair hash variant: fill and build the row table (and the pair set when b.hpairs) of b.htab.
template <typename K>
void launch_hash_rows(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, Ev ev = Ev());
template <typename K>
void launch_join_hash(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w,
                      uint32_t j, uint64_t slots, Ev ev_count = Ev(), Ev ev_emit = Ev());

// Sort *n_ptr keys of cand[0] into cand[passes & 1] in one block when they fit its LDS
// (sets ctrl->small_sorted, which turns the LSD passes of this sort into no-ops).
// `alone`: no LSD passes follow; more keys than fit set overflow bit 3 (halting the loop).
template <typename K>
void launch_small_sort(hipStream_t s, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b, int passes,
                       bool alone, Ev ev = Ev());

// Join (kind kJoinTC or kJoinSG) and sort of iteration j in one block, into cand[passes & 1]
// (the fixpoint's tail: a delta beyond one tuple per thread, or candidates beyond the
// one-block sort, set overflow bit 3).
template <typename K>
void launch_small_join(hipStream_t s, int kind, Ctrl* ctrl, const Bufs<K>& b, int w, uint32_t j, int passes,
                       Ev ev = Ev());

// The fixpoint's tail in one block (kind kJoinTC or kJoinSG): whole iterations from
// ctrl->iter + 1 on, at most up to record jmax, while they fit one block; then the
// fold of the loop's new tuples into run B (a multi-block launch; `ev_fold` times it).
template <typename K>
void launch_tail_loop(hipStream_t s, const Grid& g, int kind, Ctrl* ctrl, const Bufs<K>& b, int w, uint32_t jmax,
                      Ev ev = Ev(), Ev ev_fold = Ev());
constexpr uint32_t kTailRunBytes = 32768;  // run T of a tail loop, in LDS and in b.tail (8,192 / 4,096 keys)
constexpr uint32_t kTailKeys = 4096;       // candidates of one tail-loop iteration (sorted in LDS)
// Delta tuples a tail loop takes (its LDS: candidates, T, delta, per-tuple join state and
// the fences of A and B within the 160 KB of one workgroup): 32-bit keys 4,096 (TC) or
// 2,048 (SG), 64-bit keys 2,048 or 1,024.
constexpr uint32_t tail_tuples(size_t key_bytes, bool sg) {
  return (key_bytes == 4 ? 4096u : 2048u) >> (sg ? 1 : 0);
}

// Segmented sort of the TC join's *n_ptr candidates (grouped by row, each row's run
// unsorted) from cand[0] into cand[passes & 1]: each run sorted in LDS by one block.
// `long_rows`: runs beyond the bitonic network go to a second launch that radix-sorts
// each in LDS (up to 128 KB of keys; b.off holds the queue).  A run longer than a block
// holds sets overflow bit 4.
template <typename K>
void launch_seg_sort(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b, int w,
                     int passes, bool long_rows, Ev ev = Ev(), int gate = 0);

// One LSD pass over *n_ptr keys: pass p reads cand[p & 1] and writes cand[(p + 1) & 1];
// digit p covers bits [p * c.rb, (p + 1) * c.rb).  `scatter` false: the count and scan
// launches; true: the scatter launch.  sort_passes(key bits, c.rb) passes sort the keys,
// which end in cand[passes & 1].
template <typename K>
void launch_sort_pass(hipStream_t s, Ctrl* ctrl, const uint64_t* n_ptr, const SortCfg& c,
                      const Bufs<K>& b, int pass, bool scatter, Ev ev = Ev());

// Compaction (dedup + set difference, seeding, or the diagonal filter): local + gather.
// `in` holds *n_ptr sorted keys; `tmp` is scratch of the same capacity.
template <typename K>
void launch_compact(hipStream_t s, const Grid& g, int mode, Ctrl* ctrl, const uint64_t* n_ptr,
                    const K* in, K* tmp, const Bufs<K>& b, int w, uint32_t j, uint32_t side,
                    Ev ev = Ev(), bool narrow = false);

// Row pass of TC iteration j: the join's candidates in cand[0], grouped by row, each row
// deduplicated and set-differenced against Full in an LDS bitmap and written sorted to
// delta[j & 1] (with the gather; w <= kRowBitsMax), record j as the compaction writes it.
template <typename K>
void launch_row_diff(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b, int w,
                     uint32_t j, Ev ev = Ev(), int gate = 0);
// ... and its gather (survivors to delta[j & 1], record j); with gate 1 a row pass leaves the
// LSD passes enqueued between the two as no-ops
template <typename K>
void launch_row_gather(hipStream_t s, const Grid& g, Ctrl* ctrl, const uint64_t* n_ptr, const Bufs<K>& b,
                       uint32_t j, Ev ev = Ev(), int gate = 0);

// Merge of iteration j: B' = merge(B, delta), or on a fold A' = merge(A, B) and B' = delta.
template <typename K>
void launch_merge(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, uint32_t j,
                  Ev ev = Ev());

// O = merge(A, B) of two disjoint sorted arrays with sizes known on the host.
template <typename K>
void launch_merge_pair(hipStream_t s, const Grid& g, const K* A, uint64_t na, const K* B, uint64_t nb,
                       K* O, Ev ev = Ev());

// Edge index of the sorted, deduplicated E: Edst, and the rows (dense index when b.dense).
template <typename K>
void launch_edge_index(hipStream_t s, const Grid& g, Ctrl* ctrl, const Bufs<K>& b, int w,
                       Ev ev = Ev());

// Split keys into src / dst arrays; with n2 > 0 the keys are the union of two disjoint
// sorted runs, merged on the way.
template <typename K>
void launch_unpack(hipStream_t s, const Grid& g, const K* keys, uint64_t n, const K* keys2, uint64_t n2, int w,
                   uint32_t* src, uint32_t* dst);

void launch_resume(hipStream_t s, Ctrl* ctrl, uint64_t cand_cap, uint64_t full_cap,
                   uint32_t clear_hook);

// *ctrl = v, in stream order (v travels as the kernel argument).
void launch_ctrl_set(hipStream_t s, Ctrl* ctrl, const Ctrl& v);

}  // namespace wg
