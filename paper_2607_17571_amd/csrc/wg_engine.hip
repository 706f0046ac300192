// Host side of the fixpoint engine: buffers, the prepare phase, the batched
// device-resident loop and the C ABI declared in include/wg.h.
//
// Engine rule (Section V): the host decides when the fixpoint terminates, the device
// decides every stage size.  The host enqueues K iterations at a time, passing each
// kernel its iteration number j; every size comes from the device-side per-iteration
// records.  The host reads the control block back once per batch while a short
// speculative batch keeps the device busy (double-buffered submission, Section V-B), and
// adapts K by the paper's halving rule.

#include <algorithm>
#include <chrono>
#include <functional>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wg.h"
#include "wg_internal.h"
#include "wg_launch.h"

using namespace wg;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// What the host reads back at a batch boundary.
struct Readback {
  Ctrl c;
  IterRec first;  // record before the batch's first iteration
  IterRec last;   // record of the batch's last iteration
};

constexpr uint64_t kMaxKeys = 0xFFFFFFF0ull;  // slab offsets are 32-bit
constexpr uint32_t kMaxEvents = 1u << 16;
constexpr uint32_t kSpec = 4;                 // speculative iterations behind each batch (<= K)
constexpr uint32_t kAutoK = 2;                // iterations per host check of the default loop
constexpr uint32_t kTailIters = 512;          // iterations one tail launch may run at most
constexpr uint64_t kNarrowBelow = 1ull << 21;  // candidates below which the narrow tiles win
constexpr uint64_t kSegBelow = 1ull << 22;     // ... and the segmented sort beats the LSD passes
// kSortDual / kSortDualLsd: both routes, the row pass or the segmented sort / the LSD passes
enum : uint8_t { kSortLsd = 0, kSortSmall = 1, kSortOneBlock = 2, kSortSegmented = 3, kSortDual = 4,
                 kSortDualLsd = 5 };
// iterations expected to reach this many candidates are enqueued with both routes (the row
// pass and the segmented sort + compaction), the device picking one by kRowMin
constexpr uint64_t kDualAbove = kRowMin / 8;
constexpr uint64_t kDenseRowsMax = 1ull << 28;  // largest dense edge index (1 GB)
// fixed arrays of an engine: control block, join and compaction block totals, radix counts
// and totals (the triangle hits depend on the grid)
constexpr size_t kFixedBytes[6] = {sizeof(Ctrl), sizeof(uint64_t) * kScanBlocksMax,
                                   sizeof(uint64_t) * std::max<size_t>(kScanBlocksMax, kRowBlocks),
                                   sizeof(uint32_t) * kRadixMax * kRadixBlocksMax, sizeof(uint32_t) * kRadixMax,
                                   sizeof(uint64_t) * kRowBlocks};

thread_local std::string wg_call_error;  // see set_call_error

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct wg_engine {
  int device = 0;
  Grid grid{};
  // device memory of every engine buffer: the caller's allocator, or (has_alloc false)
  // stream-ordered hipMallocAsync / hipFreeAsync
  wg_allocator alloc{};
  bool has_alloc = false;
  Ctrl* d_ctrl = nullptr;
  Readback* h_rb = nullptr;    // pinned readback, 2 slots + 1 for stage probes
  IterRec* h_rec = nullptr;    // pinned mirror of the records, filled by the batch readbacks
  uint64_t h_rec_cap = 0;
  uint32_t rb_first[2] = {0, 0}, rb_last[2] = {0, 0};  // records each readback slot covers
  hipEvent_t ev_batch[2] = {nullptr, nullptr};
  hipEvent_t ev_done = nullptr;  // after the last launch of the latest solve (which may still
                                 // be draining its speculative batch)
  bool done_pending = false;
  uint64_t* d_jtot = nullptr;
  uint64_t* d_bcnt = nullptr;
  uint64_t* d_bstart = nullptr;  // row pass: output start of each block
  uint32_t* d_rcnt = nullptr;
  uint32_t* d_rtot = nullptr;
  uint64_t* d_hits = nullptr;  // triangle probe: hits per emit block (grid.stream entries)
  uint64_t tri_count = 0;      // the latest triangle count
  DevBuf cand[2], full[2], fullB[2], delta[2], E, U, R, Edst, rowa, rowb, off, rec, htab, tailrun;
  uint64_t hash_slots = 0;  // hash-join variant: table slots of the current solve (0: off)
  uint32_t hrows_mask = 0;  // fair hash variant: row-table slots - 1 (0: off)
  uint32_t hpairs_mask = 0; // ... and pair-set slots - 1 (triangles; 0: none)
  uint64_t dense_rows = 0;  // rows of the dense edge index of the current solve (0: U + search)
  // how the loop's iterations join and sort: 0 the LSD passes; 1 the one-block sort,
  // then the passes (no-ops when it fit); 2 the one-block sort alone; 3 the join and the
  // sort in one block (in 2 and 3 a miss halts the loop and the iteration is re-run with
  // mode 1)
  int small_mode = 1;
  // TC: the loop sorts each row's run of the grouped candidates (segmented sort) instead
  // of the LSD passes
  bool seg_sort = false;
  bool seg_long = false;  // the segmented sort hands long rows to its LDS radix pass
  // TC: the loop's iterations are enqueued with both routes -- the row pass (sort, dedup and
  // difference per row in an LDS bitmap) and the segmented sort + compaction -- and the
  // device takes the row pass from kRowMin candidates on
  bool row_bitmap = false;
  // how each iteration of the solve sorted its candidates (the method of its last
  // enqueue): kSortLsd, kSortSmall (one-block sort alone), kSortOneBlock (join and sort in
  // one block), kSortSegmented
  std::vector<uint8_t> iter_sort;
  // the loop's emit and compaction use the narrow tiles (the iterations ahead are expected
  // to have fewer than kNarrowBelow candidates)
  bool narrow = false;
  hipStream_t capture_stream = nullptr;  // private stream the iteration graph is recorded on
  hipGraphExec_t graph_exec = nullptr;   // the recorded iteration (see iteration_graph)
  std::vector<uint8_t> graph_key;        // the kernel arguments it was recorded with
  uint64_t graph_builds = 0;
  bool unfused = false;     // WG_UNFUSED_DEDUP: dedup and set difference as two passes
  bool stage_sync = false;  // WG_LOOP_STAGE: host round trips inside each iteration
  size_t allocated = 0;
  size_t peak = 0;
  uint64_t budget = 0;
  GrowHook grow_hook;  // request server: asked for more budget before a solve fails
  const std::atomic<bool>* cancel = nullptr;  // request server: stop at the next host check
  std::atomic<uint64_t> seen_cand{0};         // largest candidate count read back in this solve
  uint64_t generation = 0;
  std::string err;
  // per-solve
  uint32_t key_bytes = 4;
  int key_bits = 32;
  uint32_t num_inst = 0;                 // batched solve: instances (0: single instance)
  const uint64_t* d_offsets = nullptr;   // batched solve: edge offsets of the instances
  const SortCfg* trial = nullptr;        // autotuner: configuration under test
  SortCfg sort{};            // sort configuration of the current solve
  SortCfg tune[2];           // per key type (32-bit, 64-bit): defaults or autotuned
  uint64_t cand_cap = 0, full_cap = 0, edge_cap = 0, row_cap = 0, rec_cap = 0;
  uint64_t syncs = 0;
  // stage timing
  bool timing = false;
  uint32_t timing_mask = 0;
  std::vector<hipEvent_t> events;
  std::vector<int> event_kind;  // stage kind of each timed launch group
  uint32_t n_events = 0;         // timed launch groups (two events each)
  hipStream_t stream = nullptr;
  // result of the latest solve
  const void* res_keys = nullptr;   // the result: res_n keys, the union of two sorted runs
  uint64_t res_n = 0;
  const void* res_keys2 = nullptr;  // second run: the last res_n2 of the res_n keys
  uint64_t res_n2 = 0;
  int res_w = 16;
};

struct wg_result {
  wg_engine* engine;  // engine whose buffers hold the keys (nullptr: `owned` holds them)
  uint64_t generation;
  uint64_t n;
  int w;
  uint32_t key_bytes;
  const void* keys;
  uint32_t num_inst;  // instances (1 for a single solve)
  // the keys are the union of two disjoint sorted runs: keys[0, n - n2) and keys2[0, n2)
  const void* keys2 = nullptr;
  uint64_t n2 = 0;
  // results detached from their engine (request server)
  void* owned = nullptr;
  uint64_t owned_bytes = 0;
  // reads of an owned result enqueued on callers' streams (copies, offsets): the free waits
  // for every one of them
  mutable std::vector<hipEvent_t> uses;
  int device = 0;
  Grid grid{};
  std::function<void(uint64_t)> release;
};

namespace {

struct Fail {
  wg_status st;
};

void hip_check(wg_engine* e, hipError_t r, const char* what) {
  if (r != hipSuccess) {
    e->err = std::string(what) + ": " + hipGetErrorString(r);
    throw Fail{WG_ERR_DEVICE};
  }
}

void fail(wg_engine* e, wg_status st, const std::string& msg) {
  e->err = msg;
  throw Fail{st};
}

// Device memory of the engine, in stream order on `s`: the caller's allocator when one was
// given at creation, else the device's stream-ordered pool (hipMallocAsync), so that a
// buffer grown or freed mid-solve waits for nothing but its own stream (a plain hipFree
// would wait for the whole device).
void* dev_alloc(wg_engine* e, size_t bytes, hipStream_t s) {
  if (e->has_alloc) return e->alloc.alloc(bytes, s, e->alloc.user);
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(wg_engine* e, void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (e->has_alloc) e->alloc.free(p, bytes, s, e->alloc.user);
  else (void)hipFreeAsync(p, s);
}

void free_buf(wg_engine* e, DevBuf& b) {
  if (b.p) {
    dev_free(e, b.p, b.bytes, e->stream);
    e->allocated -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

void alloc_buf(wg_engine* e, DevBuf& b, size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  if (e->budget && e->allocated + bytes > e->budget) {
    const uint64_t granted = e->grow_hook ? e->grow_hook(e->allocated + bytes) : 0;
    if (granted < e->allocated + bytes) fail(e, WG_ERR_CAPACITY, "device memory budget exceeded");
    e->budget = granted;
  }
  void* p = dev_alloc(e, bytes, e->stream);
  if (!p) fail(e, WG_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) + " bytes failed");
  b.p = p;
  b.bytes = bytes;
  e->allocated += bytes;
  e->peak = std::max(e->peak, e->allocated);
}

// Ensure capacity without keeping contents.
void ensure(wg_engine* e, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return;
  free_buf(e, b);
  alloc_buf(e, b, bytes);
}

void sync_stream(wg_engine* e) {
  hip_check(e, hipStreamSynchronize(e->stream), "hipStreamSynchronize");
  ++e->syncs;
}

// Grow keeping the first `live` bytes.  The copy is waited for before the old buffer is
// freed, so no buffer is ever released with a read of it still pending (growth is rare).
void grow_keep(wg_engine* e, DevBuf& b, size_t bytes, size_t live) {
  if (b.bytes >= bytes && b.p) return;
  DevBuf nb;
  alloc_buf(e, nb, bytes);
  if (live && b.p) hip_check(e, hipMemcpyAsync(nb.p, b.p, live, hipMemcpyDeviceToDevice, e->stream), "copy");
  sync_stream(e);
  free_buf(e, b);
  b = nb;
}

// (Re)size every buffer for the current capacities.  With `iter`/`last`, the Full and
// delta contents that iteration iter + 1 reads (side iter & 1) are kept (grow-and-resume).
void size_buffers(wg_engine* e, bool keep, uint32_t iter, const IterRec* last) {
  const uint64_t kb = e->key_bytes;
  for (int s = 0; s < 2; ++s) ensure(e, e->cand[s], e->cand_cap * kb);
  // with `keep`: iteration iter + 1 reads run A (side last->a), run B (side last->b) and
  // the delta (side iter & 1); their contents survive the growth
  for (int s = 0; s < 2; ++s) {
    if (keep && (uint32_t)s == last->a) grow_keep(e, e->full[s], e->full_cap * kb, last->FA * kb);
    else ensure(e, e->full[s], e->full_cap * kb);
    if (keep && (uint32_t)s == last->b)
      grow_keep(e, e->fullB[s], e->full_cap * kb, (last->F - last->FA) * kb);
    else ensure(e, e->fullB[s], e->full_cap * kb);
    if (keep && (uint32_t)s == (iter & 1u)) grow_keep(e, e->delta[s], e->cand_cap * kb, last->N * kb);
    else ensure(e, e->delta[s], e->cand_cap * kb);
  }
  ensure(e, e->E, e->edge_cap * kb);
  ensure(e, e->U, (e->edge_cap + 1) * 4);
  ensure(e, e->R, (e->edge_cap + 2) * 4);
  ensure(e, e->Edst, e->edge_cap * 4);
  e->row_cap = std::max(e->cand_cap, e->edge_cap + 1);
  ensure(e, e->rowa, e->row_cap * 4);
  ensure(e, e->rowb, e->row_cap * 4);
  ensure(e, e->off, e->row_cap * 4);
  ensure(e, e->tailrun, kTailRunBytes);
}

// Free every relation buffer (the engine stays usable; the next solve starts small).
void release_relations(wg_engine* e) {
  if (e->stream) hip_check(e, hipStreamSynchronize(e->stream), "hipStreamSynchronize");
  for (int s = 0; s < 2; ++s) {
    free_buf(e, e->cand[s]);
    free_buf(e, e->full[s]);
    free_buf(e, e->fullB[s]);
    free_buf(e, e->delta[s]);
  }
  for (DevBuf* b : {&e->E, &e->U, &e->R, &e->Edst, &e->rowa, &e->rowb, &e->off, &e->rec, &e->htab, &e->tailrun})
    free_buf(e, *b);
  e->cand_cap = e->full_cap = e->edge_cap = e->row_cap = e->rec_cap = 0;
}

void ensure_records(wg_engine* e, uint64_t need) {
  if (e->rec_cap >= need) return;
  const uint64_t cap = std::max<uint64_t>(e->rec_cap * 2, need + 1024);
  DevBuf nb;
  alloc_buf(e, nb, cap * sizeof(IterRec));
  hip_check(e, hipMemsetAsync(nb.p, 0, cap * sizeof(IterRec), e->stream), "memset");
  if (e->rec.p)
    hip_check(e, hipMemcpyAsync(nb.p, e->rec.p, e->rec_cap * sizeof(IterRec), hipMemcpyDeviceToDevice,
                                e->stream), "copy");
  sync_stream(e);
  free_buf(e, e->rec);
  e->rec = nb;
  e->rec_cap = cap;
  if (e->h_rec_cap < cap) {  // the stream is drained: no readback is writing the old mirror
    IterRec* h = nullptr;
    hip_check(e, hipHostMalloc((void**)&h, cap * sizeof(IterRec)), "hipHostMalloc");
    std::memset(h, 0, cap * sizeof(IterRec));
    if (e->h_rec) {
      std::memcpy(h, e->h_rec, e->h_rec_cap * sizeof(IterRec));
      (void)hipHostFree(e->h_rec);
    }
    e->h_rec = h;
    e->h_rec_cap = cap;
  }
}

template <typename K>
Bufs<K> make_bufs(wg_engine* e) {
  Bufs<K> b;
  std::memset(&b, 0, sizeof(b));  // padding too: the bytes key the recorded iteration graph
  for (int s = 0; s < 2; ++s) {
    b.cand[s] = (K*)e->cand[s].p;
    b.full[s] = (K*)e->full[s].p;
    b.fullB[s] = (K*)e->fullB[s].p;
    b.delta[s] = (K*)e->delta[s].p;
  }
  b.E = (K*)e->E.p;
  b.U = (uint32_t*)e->U.p;
  b.R = (uint32_t*)e->R.p;
  b.Edst = (uint32_t*)e->Edst.p;
  b.rowa = (uint32_t*)e->rowa.p;
  b.rowb = (uint32_t*)e->rowb.p;
  b.off = (uint32_t*)e->off.p;
  b.jtot = e->d_jtot;
  b.bcnt = e->d_bcnt;
  b.bstart = e->d_bstart;
  b.rcnt = e->d_rcnt;
  b.rtot = e->d_rtot;
  b.hits = e->d_hits;
  b.htab = (uint64_t*)e->htab.p;
  b.hrows = e->hrows_mask;
  b.hpairs = e->hpairs_mask;
  b.rec = (IterRec*)e->rec.p;
  b.tail = (K*)e->tailrun.p;
  b.dense = (uint32_t)e->dense_rows;
  return b;
}

// ----- stage timing: events bracket launches (begin, end) when WG_STAGE_TIMING is set.
hipEvent_t pooled_event(wg_engine* e, uint32_t i) {
  while (e->events.size() <= i) {
    hipEvent_t ev;
    hip_check(e, hipEventCreate(&ev), "hipEventCreate");
    e->events.push_back(ev);
  }
  return e->events[i];
}

// Events for one launch group of stage `kind` (empty when that kind is not timed): the
// first kernel of the group stamps the start, the last the stop (hipExtLaunchKernelGGL).
Ev stage(wg_engine* e, int kind) {
  if (!e->timing || !((e->timing_mask >> kind) & 1u) || 2 * (e->n_events + 1) > kMaxEvents) return Ev();
  Ev ev;
  ev.start = pooled_event(e, 2 * e->n_events);
  ev.stop = pooled_event(e, 2 * e->n_events + 1);
  if (e->event_kind.size() <= e->n_events) e->event_kind.resize(e->n_events + 1);
  e->event_kind[e->n_events] = kind;
  ++e->n_events;
  return ev;
}

void collect_timing(wg_engine* e, wg_stats* st) {
  if (!e->timing || e->n_events == 0) return;
  hip_check(e, hipStreamSynchronize(e->stream), "hipStreamSynchronize");
  for (uint32_t i = 0; i < e->n_events; ++i) {
    float ms = 0.f;
    hip_check(e, hipEventElapsedTime(&ms, e->events[2 * i], e->events[2 * i + 1]), "hipEventElapsedTime");
    st->stage_ms[e->event_kind[i]] += ms;
    st->stage_launches[e->event_kind[i]] += 1;
  }
}

// ----- pipeline pieces
// `small` 1: the input may fit one block (then the one-block sort runs first and, if it
// did fit, the passes below exit at once); 2: it is expected to fit and the passes are not
// enqueued (a miss sets overflow bit 3); 0: the passes alone.
template <typename K>
void enqueue_sort(wg_engine* e, const Bufs<K>& b, const uint64_t* n_ptr, int small = 1) {
  const int passes = sort_passes(e->key_bits, e->sort.rb);
  if (small)
    launch_small_sort<K>(e->stream, e->d_ctrl, n_ptr, b, passes, small == 2, stage(e, WG_STAGE_RADIX_HIST));
  if (small == 2) return;
  for (int p = 0; p < passes; ++p) {
    launch_sort_pass<K>(e->stream, e->d_ctrl, n_ptr, e->sort, b, p, false, stage(e, WG_STAGE_RADIX_HIST));
    launch_sort_pass<K>(e->stream, e->d_ctrl, n_ptr, e->sort, b, p, true, stage(e, WG_STAGE_RADIX_PASS));
  }
}

// WG_LOOP_STAGE: a blocking 8-byte read of a size the stream has just produced.
void stage_probe(wg_engine* e, const uint64_t* d_size) {
  hip_check(e, hipMemcpyAsync(&e->h_rb[2].c.m_in, d_size, sizeof(uint64_t), hipMemcpyDeviceToHost, e->stream),
            "stage probe");
  sync_stream(e);
}

// How the next enqueued iteration sorts its candidates (see iter_sort).
uint8_t sort_method(const wg_engine* e, int kind) {
  if (e->small_mode == 3 && !e->hash_slots && !e->hrows_mask && !e->stage_sync) return kSortOneBlock;
  if (e->small_mode == 2) return kSortSmall;
  if (e->row_bitmap && kind == kJoinTC && !e->hash_slots) return e->seg_sort ? kSortDual : kSortDualLsd;
  if (e->seg_sort && kind == kJoinTC && !e->hash_slots) return kSortSegmented;
  return kSortLsd;
}

// One semi-naive iteration.  The kernels take the iteration number from the device
// (kIterDevice), so this launch sequence is the same for every iteration; `j` is the
// host's count, used only by the per-stage probes.
template <typename K>
void enqueue_iteration(wg_engine* e, const Bufs<K>& b, int kind, int w, int passes, uint32_t j) {
  const uint32_t jd = kIterDevice;
  const uint64_t* C = &e->d_ctrl->cand_n;
  const uint8_t method = sort_method(e, kind);
  const bool one_block = method == kSortOneBlock;
  if (one_block) {
    launch_small_join<K>(e->stream, kind, e->d_ctrl, b, w, jd, passes, stage(e, WG_STAGE_JOIN_EMIT));
  } else if (e->hash_slots) {
    const Ev ec = stage(e, WG_STAGE_JOIN_COUNT);
    launch_join_hash<K>(e->stream, e->grid, kind, e->d_ctrl, b, w, jd, e->hash_slots, ec,
                        stage(e, WG_STAGE_JOIN_EMIT));
  } else {
    launch_join_count<K>(e->stream, e->grid, kind, e->d_ctrl, b, w, jd, stage(e, WG_STAGE_JOIN_COUNT));
    launch_join_emit<K>(e->stream, e->grid, kind, e->d_ctrl, b, w, jd, stage(e, WG_STAGE_JOIN_EMIT),
                        e->narrow);
  }
  if (e->stage_sync) stage_probe(e, &b.rec[j].C);
  if (method == kSortDual || method == kSortDualLsd) {
    // both routes, gated on the join's candidate count: the row pass (sort, dedup and
    // difference of each row in one pass over cand[0]), or the sort the host picked for
    // this size (segmented, or the LSD passes, which a row pass turns into no-ops) and the
    // compaction
    launch_row_diff<K>(e->stream, e->grid, e->d_ctrl, C, b, w, jd, stage(e, WG_STAGE_ROW_DIFF), 1);
    if (method == kSortDual) {
      launch_seg_sort<K>(e->stream, e->grid, e->d_ctrl, C, b, w, passes, e->seg_long,
                         stage(e, WG_STAGE_SEG_SORT), 2);
    } else {
      for (int pp = 0; pp < passes; ++pp) {
        launch_sort_pass<K>(e->stream, e->d_ctrl, C, e->sort, b, pp, false, stage(e, WG_STAGE_RADIX_HIST));
        launch_sort_pass<K>(e->stream, e->d_ctrl, C, e->sort, b, pp, true, stage(e, WG_STAGE_RADIX_PASS));
      }
    }
    const uint32_t ps = (uint32_t)passes & 1u;
    launch_compact<K>(e->stream, e->grid, kModeIter | kModeGateSort, e->d_ctrl, C, b.cand[ps], b.cand[ps ^ 1u], b,
                      w, jd, 0, stage(e, WG_STAGE_DEDUP_DIFF), e->narrow);
    launch_row_gather<K>(e->stream, e->grid, e->d_ctrl, C, b, jd, stage(e, WG_STAGE_ROW_DIFF), 1);
    launch_merge<K>(e->stream, e->grid, e->d_ctrl, b, jd, stage(e, WG_STAGE_MERGE));
    return;
  }
  if (method == kSortSegmented)
    launch_seg_sort<K>(e->stream, e->grid, e->d_ctrl, C, b, w, passes, e->seg_long, stage(e, WG_STAGE_SEG_SORT));
  else if (!one_block)
    enqueue_sort<K>(e, b, C, std::min(e->small_mode, 2));
  const uint32_t p = (uint32_t)passes & 1u;
  if (e->unfused) {
    launch_compact<K>(e->stream, e->grid, kModeDedup, e->d_ctrl, C, b.cand[p], b.cand[p ^ 1u], b, w, jd, p,
                      stage(e, WG_STAGE_DEDUP_DIFF), e->narrow);
    launch_compact<K>(e->stream, e->grid, kModeIter, e->d_ctrl, &e->d_ctrl->dedup_n, b.cand[p],
                      b.cand[p ^ 1u], b, w, jd, 0, stage(e, WG_STAGE_DEDUP_DIFF), e->narrow);
  } else {
    launch_compact<K>(e->stream, e->grid, kModeIter, e->d_ctrl, C, b.cand[p], b.cand[p ^ 1u], b, w, jd, 0,
                      stage(e, WG_STAGE_DEDUP_DIFF), e->narrow);
  }
  if (e->stage_sync) stage_probe(e, &b.rec[j].N);
  launch_merge<K>(e->stream, e->grid, e->d_ctrl, b, jd, stage(e, WG_STAGE_MERGE));
}

// The launches of one iteration recorded once as a graph and replayed (Section V-B
// records a batch of iterations into one submission).  Recorded on a private stream and
// kept until a kernel argument changes (buffers regrown, another key type or layout).
struct IterGraphKey {
  uint8_t bufs[sizeof(Bufs<uint64_t>)];
  int kind, w, passes, key_bytes;
  SortCfg sort;
  Grid grid;
  uint64_t hash_slots;
  int unfused, small_mode, narrow, seg_sort, seg_long, row_bitmap;
};

template <typename K>
hipGraphExec_t iteration_graph(wg_engine* e, const Bufs<K>& b, int kind, int w, int passes) {
  IterGraphKey key;
  std::memset(&key, 0, sizeof(key));
  std::memcpy(key.bufs, &b, sizeof(b));
  key.kind = kind;
  key.w = w;
  key.passes = passes;
  key.key_bytes = (int)sizeof(K);
  key.sort = e->sort;
  key.grid = e->grid;
  key.hash_slots = e->hash_slots;
  key.unfused = e->unfused ? 1 : 0;
  key.small_mode = e->small_mode;
  key.narrow = e->narrow ? 1 : 0;
  key.seg_sort = e->seg_sort ? 1 : 0;
  key.seg_long = e->seg_long ? 1 : 0;
  key.row_bitmap = e->row_bitmap ? 1 : 0;
  if (e->graph_exec && e->graph_key.size() == sizeof(key) &&
      std::memcmp(e->graph_key.data(), &key, sizeof(key)) == 0)
    return e->graph_exec;
  if (e->graph_exec) {
    hip_check(e, hipGraphExecDestroy(e->graph_exec), "hipGraphExecDestroy");
    e->graph_exec = nullptr;
  }
  if (!e->capture_stream)
    hip_check(e, hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
  hipStream_t user = e->stream;
  e->stream = e->capture_stream;
  hipGraph_t g = nullptr;
  hipError_t r = hipStreamBeginCapture(e->capture_stream, hipStreamCaptureModeThreadLocal);
  if (r == hipSuccess) {
    enqueue_iteration<K>(e, b, kind, w, passes, 0);
    r = hipStreamEndCapture(e->capture_stream, &g);
  }
  e->stream = user;
  hip_check(e, r, "graph capture");
  hipGraphExec_t x = nullptr;
  r = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e, r, "hipGraphInstantiate");
  e->graph_exec = x;
  e->graph_key.assign((const uint8_t*)&key, (const uint8_t*)&key + sizeof(key));
  ++e->graph_builds;
  return x;
}

// Enqueue the readback of the control block and of records first..last (into the host
// mirror at the same indices).
void read_back(wg_engine* e, int slot, uint32_t first, uint32_t last) {
  Readback* rb = &e->h_rb[slot];
  hip_check(e, hipMemcpyAsync(&rb->c, e->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, e->stream), "readback");
  const IterRec* rec = (const IterRec*)e->rec.p;
  hip_check(e, hipMemcpyAsync(e->h_rec + first, rec + first, (size_t)(last - first + 1) * sizeof(IterRec),
                              hipMemcpyDeviceToHost, e->stream), "readback");
  hip_check(e, hipEventRecord(e->ev_batch[slot], e->stream), "hipEventRecord");
  e->rb_first[slot] = first;
  e->rb_last[slot] = last;
}

Readback wait_back(wg_engine* e, int slot) {
  hip_check(e, hipEventSynchronize(e->ev_batch[slot]), "hipEventSynchronize");
  ++e->syncs;
  Readback r = e->h_rb[slot];
  r.first = e->h_rec[e->rb_first[slot]];
  r.last = e->h_rec[e->rb_last[slot]];
  return r;
}

// Synchronous read of one record (used only with the stream drained).
IterRec read_record(wg_engine* e, uint32_t j) {
  IterRec r{};
  hip_check(e, hipMemcpyAsync(&e->h_rb[0].last, (const IterRec*)e->rec.p + j, sizeof(IterRec),
                              hipMemcpyDeviceToHost, e->stream), "record");
  sync_stream(e);
  r = e->h_rb[0].last;
  return r;
}

// Grow the buffers after an overflow and clear the flag; the loop then resumes at
// iteration c.iter + 1, whose inputs (record c.iter, its Full and delta) are intact.
void grow_and_resume(wg_engine* e, const Ctrl& c, bool hooked) {
  const IterRec last = read_record(e, c.iter);
  const IterRec next = read_record(e, c.iter + 1);
  uint64_t cand = e->cand_cap, full = e->full_cap;
  bool clear_hook = false;
  if (c.overflow & 1u) {
    if (hooked && next.C <= e->cand_cap) clear_hook = true;  // forced by the test hook
    else cand = std::max(cand * 2, next.C + next.C / 4);
  }
  if (c.overflow & 4u) cand = std::max(cand * 2, next.N + next.N / 4);
  if (c.overflow & 2u) full = std::max(full * 2, (last.F + next.N) + (last.F + next.N) / 4);
  if (cand > kMaxKeys || full > kMaxKeys)
    fail(e, WG_ERR_CAPACITY, "relation exceeds 2^32 keys per buffer");
  e->cand_cap = cand;
  e->full_cap = full;
  size_buffers(e, true, c.iter, &last);
  launch_resume(e->stream, e->d_ctrl, e->cand_cap, e->full_cap, clear_hook ? 1u : 0u);
}

// Radix field width: the bit length of the largest id.  Section V-C rounds it up to 16, 24
// or 32, a whole number of its 8-bit digits; the exact width drops bits that are zero in
// every key, which saves a pass whenever the key width crosses a digit boundary (SG on
// ER n = 500,000: 38-bit instead of 48-bit keys, 5 passes instead of 6) and keeps more
// batched keys within 32 bits.
int field_bits(uint32_t maxid) {
  int w = 1;
  while (w < 32 && (maxid >> w) != 0) ++w;
  return w;
}

void add_bytes(wg_stats* st, int k, double b) { st->stage_bytes[k] += (uint64_t)b; }

// Algorithmic HBM bytes per kernel kind (what each stage must stream at minimum).
// Algorithmic bytes: what each kernel kind must move, per launch, for the sizes the
// records hold (probes into cache-resident indexes are not counted).
//   join count  D * (kb + 4)           read delta, write one offset per tuple
//   join emit   D * (kb + 4) + C * (4 + kb) TC,  + C * (8 + kb) SG
//                                      read delta and offsets, read E.dst, write candidates
//   radix count C * kb per pass         read every key
//   radix pass  2 * C * kb per pass     read and write every key (the scatter)
//   dedup/diff  (C + N) * kb            read candidates, write the new delta
//   merge       2 * (|B| + N) * kb      read run B and the delta, write B'
//               2 * (F + N) * kb         on a fold: A and B into A', the delta into B'
//               + 2 * F * kb             once, before the SG diagonal filter: the union of
//                                        A and B (otherwise the result stays two runs,
//                                        merged by wg_result_copy)
void bytes_model(wg_stats* st, int query, uint32_t kb, int passes, uint64_t m,
                 const std::vector<IterRec>& rec, const std::vector<uint8_t>& how, uint64_t mu,
                 bool final_union) {
  // prepare: max scan (8m), pack (8m read + kb*m write), edge index (read E, write U/R/Edst)
  add_bytes(st, WG_STAGE_PREPARE, 8.0 * m + (8.0 + kb) * m + (kb + 12.0) * mu);
  add_bytes(st, WG_STAGE_RADIX_HIST, 1.0 * kb * m * passes);
  add_bytes(st, WG_STAGE_RADIX_PASS, 2.0 * kb * m * passes);
  add_bytes(st, WG_STAGE_DEDUP_DIFF, (double)kb * (m + mu));
  if (query == WG_QUERY_SG) {
    const double c = (double)rec[0].C, n = (double)rec[0].N;
    add_bytes(st, WG_STAGE_JOIN_EMIT, (kb + 8.0) * c);
    add_bytes(st, WG_STAGE_RADIX_HIST, 1.0 * kb * c * passes);
    add_bytes(st, WG_STAGE_RADIX_PASS, 2.0 * kb * c * passes);
    add_bytes(st, WG_STAGE_DEDUP_DIFF, (c + n) * kb);
  }
  const double edst = query == WG_QUERY_TC ? 4.0 : 8.0;
  for (size_t i = 1; i < rec.size(); ++i) {
    const double D = (double)rec[i - 1].N, c = (double)rec[i].C, n = (double)rec[i].N;
    const double F = (double)rec[i - 1].F;
    if (rec[i].tail) {
      // the tail loop: the edges the join reads and the delta it writes (the first delta
      // comes from HBM, the later ones stay in LDS; the probes of A and B are search
      // lines, not counted); the fold after the launch reads B and T and writes B + T
      add_bytes(st, WG_STAGE_TAIL_LOOP, c * edst + n * kb);
      if (rec[i].tail == 2) add_bytes(st, WG_STAGE_MERGE, 2.0 * (double)(rec[i].F - rec[i].FA) * kb);
      continue;
    }
    uint8_t sorted_by = i < how.size() ? how[i] : kSortLsd;
    // an iteration enqueued with both routes: the device took the rows when the join found
    // at least kRowMin candidates and Full had at most kRowFullPerCand tuples per candidate
    const bool rows = (sorted_by == kSortDual || sorted_by == kSortDualLsd) && rec[i].C >= kRowMin &&
                      rec[i].C * kRowFullPerCand >= rec[i - 1].F;
    if (sorted_by == kSortDual) sorted_by = kSortSegmented;
    if (sorted_by == kSortDualLsd) sorted_by = kSortLsd;
    if (sorted_by == kSortOneBlock) {
      // one kernel (timed as the emit): read delta and E.dst, write the sorted candidates
      add_bytes(st, WG_STAGE_JOIN_EMIT, D * kb + c * (edst + kb));
    } else if (rows) {
      // join as usual; the row pass reads the candidates and the rows of Full they touch
      // (at most all of Full) and writes the new delta, which the gather moves once more
      add_bytes(st, WG_STAGE_JOIN_COUNT, D * (kb + 4.0));
      add_bytes(st, WG_STAGE_JOIN_EMIT, D * (kb + 4.0) + c * (edst + kb));
      add_bytes(st, WG_STAGE_ROW_DIFF, (c + F + 3.0 * n) * kb);
    } else {
      add_bytes(st, WG_STAGE_JOIN_COUNT, D * (kb + 4.0));
      add_bytes(st, WG_STAGE_JOIN_EMIT, D * (kb + 4.0) + c * (edst + kb));
      if (sorted_by == kSortSegmented) {
        add_bytes(st, WG_STAGE_SEG_SORT, 2.0 * c * kb);
      } else if (sorted_by == kSortSmall) {
        add_bytes(st, WG_STAGE_RADIX_HIST, 2.0 * c * kb);
      } else {
        add_bytes(st, WG_STAGE_RADIX_HIST, 1.0 * c * kb * passes);
        add_bytes(st, WG_STAGE_RADIX_PASS, 2.0 * c * kb * passes);
      }
    }
    if (!rows) add_bytes(st, WG_STAGE_DEDUP_DIFF, (c + n) * kb);
    // the merge: delta into run B, or on a fold B into A plus the delta as the new B
    const double FA = (double)rec[i - 1].FA, FB = F - FA;
    if (rec[i].fold) add_bytes(st, WG_STAGE_MERGE, 2.0 * (FA + FB + n) * kb);
    else if (rec[i].N > 0) add_bytes(st, WG_STAGE_MERGE, 2.0 * (FB + n) * kb);
  }
  const IterRec& fin = rec.back();
  if (final_union && fin.F > fin.FA) add_bytes(st, WG_STAGE_MERGE, 2.0 * (double)fin.F * kb);
}

template <typename K>
wg_status run(wg_engine* e, int query, const uint32_t* src, const uint32_t* dst, uint64_t m,
              const wg_options& o, int w, int ib, wg_stats* st) {
  e->key_bits = ib + 2 * w;
  e->seen_cand.store(0, std::memory_order_relaxed);
  e->sort = e->trial ? *e->trial : e->tune[sizeof(K) == 8];
  if (o.radix_digit_bits) e->sort.rb = (int)o.radix_digit_bits;
  if (o.tile_items) e->sort.items = (int)o.tile_items;
  const int passes = sort_passes(e->key_bits, e->sort.rb);
  e->key_bytes = sizeof(K);
  e->edge_cap = std::max<uint64_t>(e->edge_cap, m);
  e->cand_cap = std::min(std::max<uint64_t>({e->cand_cap, 2 * m, 1u << 20}), kMaxKeys);
  e->full_cap = std::min(std::max<uint64_t>({e->full_cap, 2 * m, 1u << 20}), kMaxKeys);
  size_buffers(e, false, 0, nullptr);
  if (e->dense_rows) ensure(e, e->R, (e->dense_rows + 1) * 4);
  ensure_records(e, 1024);
  hip_check(e, hipMemsetAsync(e->rec.p, 0, e->rec_cap * sizeof(IterRec), e->stream), "memset");

  Ctrl c0;
  std::memset(&c0, 0, sizeof(Ctrl));
  c0.m_in = m;
  c0.cand_cap = e->cand_cap;
  c0.full_cap = e->full_cap;
  c0.max_iter = (uint32_t)std::min<uint64_t>(o.max_iterations, 0xFFFFFFFFu);
  c0.force_overflow_at = (uint32_t)std::min<uint64_t>(o.force_overflow_at_iter, 0xFFFFFFFFu);
  launch_ctrl_set(e->stream, e->d_ctrl, c0);

  // ---- prepare: sort + dedup E, edge index, seed (Section IV-A: E sorted once)
  // (the join variants of an earlier solve are cleared before the buffers are described)
  e->hash_slots = 0;
  e->hrows_mask = e->hpairs_mask = 0;
  Bufs<K> b = make_bufs<K>(e);
  if (e->num_inst)
    launch_pack_batch<K>(e->stream, e->grid, src, dst, m, w, e->d_offsets, e->num_inst, b.cand[0],
                         stage(e, WG_STAGE_PREPARE));
  else
    launch_pack<K>(e->stream, e->grid, src, dst, m, w, b.cand[0], stage(e, WG_STAGE_PREPARE));
  // (the m packed keys are all sorted: when they fit one block its sort runs alone)
  enqueue_sort<K>(e, b, &e->d_ctrl->m_in, m * sizeof(K) <= kSmallSortBytes ? 2 : 0);
  const int mode = query == WG_QUERY_SG ? kModeEdges : (kModeEdges | kModeSeed);
  launch_compact<K>(e->stream, e->grid, mode, e->d_ctrl, &e->d_ctrl->m_in, b.cand[passes & 1],
                    b.cand[(passes & 1) ^ 1], b, w, 0, 0, stage(e, WG_STAGE_DEDUP_DIFF));
  launch_edge_index<K>(e->stream, e->grid, e->d_ctrl, b, w, stage(e, WG_STAGE_PREPARE));
  e->unfused = (o.flags & WG_UNFUSED_DEDUP) != 0;
  e->stage_sync = false;
  if (o.flags & WG_JOIN_HASH) {
    // hash-join variant: a table of E with at least twice as many slots as edges
    uint64_t slots = 1024;
    while (slots < 2 * m) slots <<= 1;
    if (slots > (1ull << 32)) fail(e, WG_ERR_CAPACITY, "hash table beyond 2^32 slots");
    ensure(e, e->htab, slots * sizeof(uint64_t));
    e->hash_slots = slots;
    b = make_bufs<K>(e);
    launch_hash_build<K>(e->stream, e->grid, e->d_ctrl, b, w, slots, stage(e, WG_STAGE_PREPARE));
  }
  if (o.flags & WG_JOIN_HASH_ROWS) {
    // fair hash variant: a table of E's distinct rows (row -> index of its edges) and, for
    // triangles, a set of E's pairs, each with at least twice as many slots as edges
    uint64_t slots = 1024;
    while (slots < 2 * m) slots <<= 1;
    if (slots > (1ull << 31)) fail(e, WG_ERR_CAPACITY, "hash table beyond 2^31 slots");
    const uint64_t pairs = query == WG_QUERY_TRIANGLES ? slots : 0;
    ensure(e, e->htab, (slots + pairs) * sizeof(uint64_t));
    e->hrows_mask = (uint32_t)(slots - 1);
    e->hpairs_mask = pairs ? (uint32_t)(pairs - 1) : 0u;
    b = make_bufs<K>(e);
    launch_hash_rows<K>(e->stream, e->grid, e->d_ctrl, b, stage(e, WG_STAGE_PREPARE));
  }

  if (query == WG_QUERY_TRIANGLES) {
    // Section VI: one pass of the join of E with itself; the emit phase probes E for the
    // closing edge of each two-path and counts the hits per block
    if (e->hash_slots) {
      const Ev ec = stage(e, WG_STAGE_JOIN_COUNT);
      launch_join_hash<K>(e->stream, e->grid, kJoinTri, e->d_ctrl, b, w, 1, e->hash_slots, ec,
                          stage(e, WG_STAGE_JOIN_EMIT));
    } else {
      launch_join_count<K>(e->stream, e->grid, kJoinTri, e->d_ctrl, b, w, 1, stage(e, WG_STAGE_JOIN_COUNT));
      launch_join_emit<K>(e->stream, e->grid, kJoinTri, e->d_ctrl, b, w, 1, stage(e, WG_STAGE_JOIN_EMIT));
    }
    // the sorted probe writes one total per emit block (grid.stream), the hash probe one
    // per count block (grid.scan)
    std::vector<uint64_t> hits((size_t)(e->hash_slots ? e->grid.scan : e->grid.stream));
    hip_check(e, hipMemcpyAsync(hits.data(), e->d_hits, hits.size() * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, e->stream), "readback");
    read_back(e, 0, 0, 1);
    const Readback r = wait_back(e, 0);
    if (r.c.overflow) fail(e, WG_ERR_CAPACITY, "more than 2^32 two-paths");
    uint64_t total = 0;
    for (uint64_t h : hits) total += h;
    e->tri_count = total;
    e->res_keys = e->res_keys2 = nullptr;
    e->res_n = e->res_n2 = 0;
    e->res_w = w;
    if (st) {
      st->iterations = 1;
      st->base_tuples = r.first.N;
      st->join_candidates = r.last.C;
      st->field_bits = (uint32_t)w;
      st->key_bytes = (uint32_t)sizeof(K);
      st->digit_bits = (uint32_t)e->sort.rb;
      st->sort_passes = (uint32_t)passes;
      const double D = (double)r.first.N, C = (double)r.last.C;
      add_bytes(st, WG_STAGE_JOIN_COUNT, D * (sizeof(K) + 4.0));
      add_bytes(st, WG_STAGE_JOIN_EMIT, D * (sizeof(K) + 4.0) + C * 4.0);
      collect_timing(e, st);
    }
    return WG_OK;
  }

  uint64_t seed_n = m;  // |Delta^0| (TC: at most m; SG: read back below)
  if (query == WG_QUERY_SG) {
    // base rule: Delta^0 = Full = {(x, y) : E(p, x), E(p, y), x != y}, sorted + deduplicated
    for (;;) {
      b = make_bufs<K>(e);
      launch_join_count<K>(e->stream, e->grid, kJoinSGBase, e->d_ctrl, b, w, 0, stage(e, WG_STAGE_JOIN_COUNT));
      launch_join_emit<K>(e->stream, e->grid, kJoinSGBase, e->d_ctrl, b, w, 0, stage(e, WG_STAGE_JOIN_EMIT));
      enqueue_sort<K>(e, b, &b.rec[0].C);
      launch_compact<K>(e->stream, e->grid, kModeSeed, e->d_ctrl, &b.rec[0].C, b.cand[passes & 1],
                        b.cand[(passes & 1) ^ 1], b, w, 0, 0, stage(e, WG_STAGE_DEDUP_DIFF));
      read_back(e, 0, 0, 0);
      const Readback r = wait_back(e, 0);
      seed_n = r.last.N;
      if (!r.c.overflow) break;
      if (r.c.overflow & 1u) e->cand_cap = std::max(e->cand_cap * 2, r.last.C + r.last.C / 4);
      if (r.c.overflow & 2u) {
        const uint64_t need = r.last.N > 0 ? r.last.N : r.last.C;
        e->full_cap = std::max(e->full_cap * 2, need + need / 4);
        e->cand_cap = std::max(e->cand_cap, need + need / 4);
      }
      if (e->cand_cap > kMaxKeys || e->full_cap > kMaxKeys)
        fail(e, WG_ERR_CAPACITY, "relation exceeds 2^32 keys per buffer");
      sync_stream(e);
      size_buffers(e, false, 0, nullptr);
      launch_resume(e->stream, e->d_ctrl, e->cand_cap, e->full_cap, 0);
      if (st) st->resumes++;
    }
  }

  // ---- the semi-naive loop, K iterations per host check
  const int kind = query == WG_QUERY_TC ? kJoinTC : kJoinSG;
  // Section V-B sizes batches for a host round trip of milliseconds: K = 30 halving for
  // TC, 10 for SG (WG_LOOP_BATCHED with batch_k = 0).  Here a round trip costs about
  // 12 us and the speculative batch hides it, while every iteration enqueued past the
  // fixpoint still costs its no-op launches (about 30 us), so the default checks every
  // kAutoK iterations.
  const bool paper_policy = o.loop_mode == WG_LOOP_BATCHED && o.batch_k == 0;
  uint32_t K_batch = o.batch_k ? o.batch_k : (paper_policy ? (query == WG_QUERY_TC ? 30u : 10u) : kAutoK);
  const bool adaptive = paper_policy && query == WG_QUERY_TC;
  if (o.loop_mode == WG_LOOP_HOST || o.loop_mode == WG_LOOP_STAGE) K_batch = 1;
  const bool speculate = !(o.flags & WG_NO_SPECULATION) && o.loop_mode != WG_LOOP_STAGE;
  e->stage_sync = o.loop_mode == WG_LOOP_STAGE;
  const bool hooked = o.force_overflow_at_iter != 0;
  uint32_t next_j = 1;
  uint32_t batch_first = 1;
  Readback r{};
  int slot = 0;
  // WG_ITER_GRAPH replays the recorded iteration; the event-timed and per-stage-probed
  // loops always launch one by one
  const bool graphs = !e->timing && !e->stage_sync && (o.flags & WG_ITER_GRAPH);
  auto enqueue_iters = [&](uint32_t k) {
    ensure_records(e, (uint64_t)next_j + k + 2);
    b = make_bufs<K>(e);
    if (e->iter_sort.size() < (size_t)next_j + k + 1) e->iter_sort.resize((size_t)next_j + k + 1 + 64);
    for (uint32_t i = 0; i < k; ++i) e->iter_sort[next_j + i] = sort_method(e, kind);
    if (graphs && k > 0) {
      hipGraphExec_t x = iteration_graph<K>(e, b, kind, w, passes);
      for (uint32_t i = 0; i < k; ++i) {
        hip_check(e, hipGraphLaunch(x, e->stream), "hipGraphLaunch");
        ++next_j;
      }
      return;
    }
    for (uint32_t i = 0; i < k; ++i) enqueue_iteration<K>(e, b, kind, w, passes, next_j++);
  };
  auto enqueue_batch = [&](uint32_t k, int sl) {
    enqueue_iters(k);
    read_back(e, sl, batch_first - 1, next_j - 1);
    batch_first = next_j;
  };
  // The one-block sort is enqueued while the last checked iteration's candidates were
  // within 4x of what it holds (the first batch has no size yet).  Once they are at most
  // a quarter of it, or half of it and not growing, it is enqueued alone, without the LSD
  // passes behind it (a dozen no-op launches per iteration of the fixpoint's tail): the
  // loop's next iterations run up to a batch and a speculative batch ahead of that check,
  // and a miss halts the loop, which re-runs the iteration with the passes and keeps them
  // for the rest of the solve.  Batches of many iterations (the paper's policy) never go
  // alone.
  const uint64_t small_keys = kSmallSortBytes / sizeof(K);
  const uint64_t tail_n_max = tail_tuples(sizeof(K), kind == kJoinSG);
  bool tail_ok = false;  // the last check's sizes (and their rate) fit the tail loop
  bool small_missed = false;
  // within a quarter of a limit, or half of it and not growing
  bool seg_allowed = query == WG_QUERY_TC && !(o.flags & WG_LSD_SORT);
  // the row pass: one instance (at most 2^w rows, so a large iteration has long rows), ids
  // within the LDS bitmap, the fused compaction
  const bool row_allowed = seg_allowed && e->num_inst <= 1 && w <= kRowBitsMax && !e->unfused &&
                           !e->stage_sync && !e->hash_slots;
  bool long_forced = false;  // a row outgrew the bitonic network: long-row pass from now on
  auto calm = [&](uint64_t now, uint64_t before, uint64_t limit) {
    return 4 * now <= limit || (2 * now <= limit && now <= before);
  };
  auto pick_small_mode = [&](uint32_t it) {
    const IterRec& x = e->h_rec[it];
    const IterRec& y = e->h_rec[it > 0 ? it - 1 : 0];
    // narrow tiles while the candidates, grown at the last checked rate for the iterations
    // already enqueued ahead (up to a batch and a speculative batch), stay below the bound
    double g = it >= 2 && y.C > 0 ? (double)x.C / (double)y.C : 4.0;
    g = std::max(g, 1.0);
    const double ahead = (double)x.C * g * g * g * g;
    e->narrow = ahead < (double)kNarrowBelow;
    e->seg_sort = seg_allowed && ahead < (double)kSegBelow;
    // (the row route needs at least a kRowFullPerCand-th of Full's tuples as candidates, and
    // Full only grows: below that the row launches would all be gated off)
    e->row_bitmap = row_allowed && seg_allowed && ahead >= (double)kDualAbove &&
                    ahead * (double)kRowFullPerCand >= (double)x.F;
    e->seg_long = (e->seg_sort || e->row_bitmap) && long_forced;
    if (!small_missed && K_batch <= kAutoK && it >= 2 && calm(x.C, y.C, small_keys))
      e->small_mode = calm(x.N, y.N, kSmallJoinTuples) ? 3 : 2;
    else
      e->small_mode = x.C <= 4 * small_keys ? 1 : 0;
    // (the tail loop checks every iteration's sizes itself: a wrong guess costs one launch)
    tail_ok = it >= 1 && calm(x.C, y.C, kTailKeys) && calm(x.N, y.N, tail_n_max);
  };
  e->small_mode = 1;
  e->narrow = false;  // (no size yet: the first iterations can already be large)
  // TC: the segmented sort while the iterations ahead are expected below kSegBelow
  // candidates (larger ones sort faster through the LSD passes); once a row outgrows the
  // bitonic network, with the long-row pass, and once a row outgrows that pass too, the
  // LSD passes for the rest of the solve; the first batch, sizes unknown, takes the LSD
  // passes
  e->seg_sort = e->seg_long = false;
  // The tail loop (WG_LOOP_AUTO): where the delta and the candidates, at the last check
  // and at their rate of change, fit one block, the host launches one block running
  // iterations up to the fixpoint or until one outgrows it, and the fold after it, with
  // nothing behind them, and waits.  A tail loop stopped by an iteration that does not
  // fit hands that iteration to a batch.
  const bool tail_allowed = o.loop_mode == WG_LOOP_AUTO && !(o.flags & WG_NO_TAIL_LOOP) && !e->hash_slots &&
                            !e->hrows_mask && !e->unfused;
  bool in_tail = false;  // the launch waited on is a tail loop
  auto enqueue_tail = [&](int sl) {
    const uint32_t jmax = next_j + kTailIters - 1;
    ensure_records(e, (uint64_t)jmax + 2);
    b = make_bufs<K>(e);
    launch_tail_loop<K>(e->stream, e->grid, kind, e->d_ctrl, b, w, jmax, stage(e, WG_STAGE_TAIL_LOOP),
                        stage(e, WG_STAGE_MERGE));
    next_j = jmax + 1;
    read_back(e, sl, batch_first - 1, next_j - 1);
    batch_first = next_j;
  };
  // (the first batch, sizes unknown, takes both routes where the row pass is allowed)
  e->row_bitmap = row_allowed;
  if (tail_allowed && seed_n <= tail_n_max && seed_n <= kTailKeys) {
    // a small seed: the tail loop from the first iteration (it stops at once if the
    // first join is beyond it)
    enqueue_tail(slot);
    in_tail = true;
  } else {
    enqueue_batch(K_batch, slot);
  }
  for (;;) {
    // While the host waits on this batch, the device runs a short speculative batch
    // behind it (Section V-B overlaps the next batch with the host check); after the
    // fixpoint its launches are no-ops, so it is kept short.
    if (speculate && !in_tail) enqueue_iters(std::min(K_batch, kSpec));
    r = wait_back(e, slot);
    if (in_tail) {
      // nothing ran behind the tail loop: the host's count resumes from the device's
      next_j = r.c.iter + 1;
      batch_first = next_j;
    }
    if (r.c.cand_n > e->seen_cand.load(std::memory_order_relaxed))
      e->seen_cand.store(r.c.cand_n, std::memory_order_relaxed);
    const bool tail_stuck = in_tail && r.c.tail_exit == kTailSizes;
    in_tail = false;
    pick_small_mode(r.c.iter);
    if (tail_stuck && r.c.iter == 0) {
      // the first iteration was beyond the tail loop: sizes still unknown, as at the start
      e->small_mode = 1;
      e->narrow = e->seg_sort = e->seg_long = false;
      e->row_bitmap = row_allowed;
    }
    // (at the fixpoint the speculative batch still drains behind the final launches;
    // everything after this is stream-ordered and reads the host mirror of the records)
    if (r.c.overflow | r.c.limit_hit) sync_stream(e);
    if (e->cancel && e->cancel->load()) {
      sync_stream(e);
      fail(e, WG_ERR_CANCELLED, "cancelled");
    }
    if (r.c.overflow) {
      if (r.c.overflow & 8u) {
        small_missed = true;
        e->small_mode = 1;
      }
      if (r.c.overflow & 16u) {
        // the first long row turns the long-row pass on for the rest of the solve; a row
        // beyond even that pass (or a second overflow) leaves the LSD passes
        if (!long_forced) {
          long_forced = true;
          e->seg_long = e->seg_sort || e->row_bitmap;
        } else {
          seg_allowed = e->seg_sort = e->seg_long = e->row_bitmap = false;
        }
      }
      grow_and_resume(e, r.c, hooked);
      if (st) st->resumes++;
      next_j = r.c.iter + 1;
      batch_first = next_j;
      enqueue_batch(K_batch, slot);
      continue;
    }
    if (r.c.done || r.c.limit_hit) break;
    // Section V-B: halve K when the batch's last/first delta-size ratio is below 0.1
    if (adaptive && r.first.N > 0 && (double)r.last.N / (double)r.first.N < 0.1)
      K_batch = std::max(1u, K_batch / 2);
    slot ^= 1;
    if (tail_allowed && tail_ok && !tail_stuck) {
      enqueue_tail(slot);
      in_tail = true;
      continue;
    }
    // (an iteration the tail loop left over does not fit the one-block join)
    if (tail_stuck && e->small_mode == 3) e->small_mode = 1;
    enqueue_batch(K_batch, slot);
  }
  if (r.c.limit_hit && !r.c.done) fail(e, WG_ERR_ITER_LIMIT, "max_iterations reached before the fixpoint");

  // result: Full after the last iteration, the union of its runs A and B (one final
  // disjoint merge into the free A buffer unless B is empty)
  const uint32_t iters = r.c.iter;
  const IterRec fin = e->h_rec[iters];  // covered by the last readback
  uint32_t side = fin.a;
  uint64_t F = fin.F;
  b = make_bufs<K>(e);
  const bool filter = query == WG_QUERY_SG && (o.flags & WG_SG_IRREFLEXIVE) && F > 0;
  e->res_keys2 = nullptr;
  e->res_n2 = 0;
  if (fin.F > fin.FA && !filter) {
    // the result stays two runs; reading it merges them (wg_result_copy)
    e->res_keys2 = b.fullB[fin.b];
    e->res_n2 = fin.F - fin.FA;
  } else if (fin.F > fin.FA) {
    launch_merge_pair<K>(e->stream, e->grid, b.full[fin.a], fin.FA, b.fullB[fin.b], fin.F - fin.FA,
                         b.full[fin.a ^ 1u], stage(e, WG_STAGE_MERGE));
    side = fin.a ^ 1u;
  }
  if (filter) {
    if (e->cand_cap < F) {
      e->cand_cap = F;
      for (int s = 0; s < 2; ++s) ensure(e, e->cand[s], e->cand_cap * e->key_bytes);
      b = make_bufs<K>(e);
    }
    launch_compact<K>(e->stream, e->grid, kModeFilter, e->d_ctrl, &b.rec[iters].F, b.full[side],
                      b.cand[0], b, w, 0, side, stage(e, WG_STAGE_PREPARE));
    read_back(e, 0, 0, 0);
    F = wait_back(e, 0).c.filtered;
    side ^= 1u;
  }
  e->res_keys = b.full[side];
  e->res_n = F;
  e->res_w = w;

  if (st) {
    st->iterations = iters;
    st->result_tuples = F;
    st->field_bits = (uint32_t)w;
    st->key_bytes = (uint32_t)sizeof(K);
    st->digit_bits = (uint32_t)e->sort.rb;
    st->sort_passes = (uint32_t)passes;
    // every record up to the fixpoint came back with some batch readback
    const std::vector<IterRec> recs(e->h_rec, e->h_rec + iters + 1);
    st->base_tuples = recs[0].N;
    for (const IterRec& x : recs) st->tail_iterations += x.tail ? 1u : 0u;
    uint64_t cand_total = 0;
    for (size_t i = 1; i < recs.size(); ++i) cand_total += recs[i].C;
    st->join_candidates = cand_total;
    if (st->delta_sizes)
      for (uint64_t i = 0; i < std::min<uint64_t>(st->delta_sizes_cap, recs.size()); ++i)
        st->delta_sizes[i] = recs[i].N;
    bytes_model(st, query, sizeof(K), passes, m, recs, e->iter_sort, r.c.m_unique, filter);
    collect_timing(e, st);
  }
  return WG_OK;
}

bool is_device_pointer(const void* p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((1ull << b) < v) ++b;
  return b;
}

// num == 0: a single instance; else a batch of `num` instances with edge offsets.
wg_status solve(wg_engine* e, int query, uint32_t num, const uint64_t* d_offsets,
                const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* opt_in, void* stream, wg_result** out, wg_stats* st) {
  if (!e) return WG_ERR_INVALID_ARG;
  const double t0 = now_ms();
  e->err.clear();
  if (!out) {
    e->err = "out is NULL";
    return WG_ERR_INVALID_ARG;
  }
  *out = nullptr;
  wg_options o{};
  o.struct_size = sizeof(wg_options);
  if (opt_in) {
    if (opt_in->struct_size < 8 || opt_in->struct_size > sizeof(wg_options)) {
      e->err = "wg_options.struct_size is not a known size";
      return WG_ERR_INVALID_ARG;
    }
    std::memcpy(&o, opt_in, opt_in->struct_size);
  }
  if (m > 0 && (!d_src || !d_dst)) {
    e->err = "NULL edge array with m > 0";
    return WG_ERR_INVALID_ARG;
  }
  if (num > 0 && !d_offsets) {
    e->err = "NULL offsets for a batch";
    return WG_ERR_INVALID_ARG;
  }
  if (num > (1u << 24)) {
    e->err = "more than 2^24 instances";
    return WG_ERR_INVALID_ARG;
  }
  if (m >= kMaxKeys / 2) {
    e->err = "too many edges";
    return WG_ERR_INVALID_ARG;
  }
  if (o.radix_field_bits > 32) {
    e->err = "radix_field_bits must be 0..32";
    return WG_ERR_INVALID_ARG;
  }
  if (o.radix_digit_bits != 0 &&
      (o.radix_digit_bits < (uint32_t)kRadixBitsMin || o.radix_digit_bits > (uint32_t)kRadixBitsMax)) {
    e->err = "radix_digit_bits must be 0 or 8..11";
    return WG_ERR_INVALID_ARG;
  }
  if (o.tile_items != 0 && o.tile_items != 8 && o.tile_items != 12 && o.tile_items != 16) {
    e->err = "tile_items must be 0, 8, 12 or 16";
    return WG_ERR_INVALID_ARG;
  }
  if ((o.flags & (WG_JOIN_HASH | WG_JOIN_HASH_ROWS)) && query == WG_QUERY_SG) {
    e->err = "WG_JOIN_HASH and WG_JOIN_HASH_ROWS apply to TC and triangle counting";
    return WG_ERR_INVALID_ARG;
  }
  if ((o.flags & WG_JOIN_HASH) && (o.flags & WG_JOIN_HASH_ROWS)) {
    e->err = "WG_JOIN_HASH and WG_JOIN_HASH_ROWS exclude each other";
    return WG_ERR_INVALID_ARG;
  }
  if (o.loop_mode > WG_LOOP_STAGE ||
      (o.flags & ~(WG_SG_IRREFLEXIVE | WG_STAGE_TIMING | WG_NO_SPECULATION | WG_JOIN_HASH | WG_UNFUSED_DEDUP |
                   WG_SPARSE_INDEX | WG_ITER_GRAPH | WG_LSD_SORT | WG_JOIN_HASH_ROWS | WG_NO_TAIL_LOOP))) {
    e->err = "unknown loop_mode or flag";
    return WG_ERR_INVALID_ARG;
  }
  if (st) {
    uint64_t* ds = st->delta_sizes;
    uint64_t dc = st->delta_sizes_cap;
    std::memset(st, 0, sizeof(*st));
    st->delta_sizes = ds;
    st->delta_sizes_cap = dc;
  }
  try {
    hip_check(e, hipSetDevice(e->device), "hipSetDevice");
    e->stream = (hipStream_t)stream;
    // the previous solve may have returned with launches still queued on its stream:
    // this one's stream waits for them (a no-op on the same stream)
    if (e->done_pending) {
      hip_check(e, hipStreamWaitEvent(e->stream, e->ev_done, 0), "hipStreamWaitEvent");
      e->done_pending = false;
    }
    e->generation++;
    e->res_keys = e->res_keys2 = nullptr;
    e->res_n = e->res_n2 = 0;
    e->syncs = 0;
    e->budget = o.mem_budget_bytes;
    // the budget bounds everything the engine holds: buffers kept from earlier solves
    // that already exceed it are released first
    if (e->budget && e->allocated > e->budget) release_relations(e);
    e->peak = e->allocated;
    e->timing = (o.flags & WG_STAGE_TIMING) != 0;
    e->timing_mask = o.timing_stages ? o.timing_stages : 0xFFFFFFFFu;
    e->n_events = 0;
    e->num_inst = num;
    e->d_offsets = d_offsets;
    const int ib = num > 1 ? ceil_log2(num) : 0;
    if (m == 0) {
      if (st && st->delta_sizes && st->delta_sizes_cap) st->delta_sizes[0] = 0;
    } else {
      // largest id -> radix field width (Section V-C); the one synchronisation before the loop
      Ctrl zero;
      std::memset(&zero, 0, sizeof(Ctrl));
      launch_ctrl_set(e->stream, e->d_ctrl, zero);
      launch_max_id(e->stream, e->grid, e->d_ctrl, d_src, d_dst, m);
      if (num) launch_check_offsets(e->stream, e->grid, e->d_ctrl, d_offsets, num, m);
      hip_check(e, hipMemcpyAsync(&e->h_rb[0].c, e->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, e->stream),
                "readback");
      sync_stream(e);
      if (e->h_rb[0].c.bad_input) {
        e->err = "batch offsets must start at 0, not decrease and end at m";
        return WG_ERR_INVALID_ARG;
      }
      int w = field_bits(e->h_rb[0].c.maxid);
      if (o.radix_field_bits) {
        const uint32_t maxid = e->h_rb[0].c.maxid;
        if (o.radix_field_bits < 32 && (maxid >> o.radix_field_bits) != 0) {
          e->err = "radix_field_bits does not cover the largest vertex id";
          return WG_ERR_INVALID_ARG;
        }
        w = (int)o.radix_field_bits;
      }
      if (ib + w > 32) {
        e->err = "batch too wide: instance bits plus the id field exceed 32 bits";
        return WG_ERR_INVALID_ARG;
      }
      // Row ids are (instance << w) | src.  When they span a range not much larger than the
      // graph, the edge index is a dense array over that range (two loads per lookup);
      // otherwise a sorted array of the distinct rows searched by bisection.
      const uint64_t space = (num > 1 ? ((uint64_t)(num - 1) << w) : 0) + e->h_rb[0].c.maxid + 1;
      // (the fair hash variant looks rows up through its table: it keeps the rows' list)
      e->dense_rows = (!(o.flags & (WG_SPARSE_INDEX | WG_JOIN_HASH_ROWS)) && space <= kDenseRowsMax &&
                       space <= 16 * m + (1u << 20))
                          ? space
                          : 0;
      wg_status r = (ib + 2 * w <= 32) ? run<uint32_t>(e, query, d_src, d_dst, m, o, w, ib, st)
                                       : run<uint64_t>(e, query, d_src, d_dst, m, o, w, ib, st);
      if (r != WG_OK) return r;
      hip_check(e, hipEventRecord(e->ev_done, e->stream), "hipEventRecord");
      e->done_pending = true;
    }
    wg_result* res = new wg_result{e, e->generation, e->res_n, e->res_w, e->key_bytes, e->res_keys,
                                   num ? num : 1u};
    res->keys2 = e->res_keys2;
    res->n2 = e->res_n2;
    *out = res;
    if (st) {
      st->host_syncs = e->syncs;
      st->solve_ms = now_ms() - t0;
    }
    return WG_OK;
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(e->stream);
    return f.st;
  }
}

// ----- result handles: engine-backed (valid until the engine's next solve) or owned
wg_status check_result(const wg_result* r) {
  if (!r) return WG_ERR_INVALID_ARG;
  if (r->owned || r->n == 0) return WG_OK;
  if (!r->engine) return WG_ERR_INVALID_ARG;
  if (r->generation != r->engine->generation) {
    r->engine->err = "result is stale: the engine ran another solve";
    return WG_ERR_STALE;
  }
  return WG_OK;
}

void note(const wg_result* r, const char* msg) {
  if (r->engine) r->engine->err = msg;
}

wg_status device_error(const wg_result* r, const char* what) {
  const hipError_t err = hipGetLastError();
  if (r->engine) r->engine->err = std::string(what) + ": " + hipGetErrorString(err);
  return WG_ERR_DEVICE;
}

int result_device(const wg_result* r) { return r->engine ? r->engine->device : r->device; }

// Reads of an engine-backed result on stream s: they wait for the solve's launches (which
// may still be queued on the solve's stream), and the engine's next solve, on any stream,
// waits for them before reusing the buffers.
hipError_t wait_engine(const wg_result* r, hipStream_t s) {
  if (!r->engine || !r->engine->done_pending) return hipSuccess;
  return hipStreamWaitEvent(s, r->engine->ev_done, 0);
}

hipError_t mark_engine_use(const wg_result* r, hipStream_t s) {
  if (!r->engine) {
    // an owned result: its free must come after this read, whatever stream it is on
    hipEvent_t ev = nullptr;
    hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(ev, s);
    if (ev) r->uses.push_back(ev);
    return err;
  }
  const hipError_t err = hipEventRecord(r->engine->ev_done, s);
  if (err == hipSuccess) r->engine->done_pending = true;
  return err;
}
Grid result_grid(const wg_result* r) { return r->engine ? r->engine->grid : r->grid; }

}  // namespace

namespace wg {

wg_status engine_solve(wg_engine* e, int query, uint32_t num, const uint64_t* d_offsets,
                       const uint32_t* src, const uint32_t* dst, uint64_t m, const wg_options* o,
                       void* stream, wg_result** out, wg_stats* st) {
  return solve(e, query, num, d_offsets, src, dst, m, o, stream, out, st);
}

void set_call_error(const char* msg) { wg_call_error = msg; }

uint64_t engine_allocated(const wg_engine* e) { return e->allocated; }
uint64_t engine_peak(const wg_engine* e) { return e->peak; }
void engine_set_grow_hook(wg_engine* e, GrowHook hook) { e->grow_hook = std::move(hook); }
void engine_set_cancel(wg_engine* e, const std::atomic<bool>* flag) { e->cancel = flag; }
uint64_t engine_seen_candidates(const wg_engine* e) { return e->seen_cand.load(std::memory_order_relaxed); }
void engine_clear_seen(wg_engine* e) { e->seen_cand.store(0, std::memory_order_relaxed); }

void engine_trim(wg_engine* e) {
  try {
    hip_check(e, hipSetDevice(e->device), "hipSetDevice");
    release_relations(e);
  } catch (const Fail&) {
  }
  e->generation++;
  e->res_keys = e->res_keys2 = nullptr;
  e->res_n = e->res_n2 = 0;
}

wg_status result_detach(const wg_result* r, hipStream_t s, std::function<void(uint64_t)> release,
                        wg_result** out, uint64_t* bytes) {
  const wg_status v = check_result(r);
  if (v != WG_OK) return v;
  wg_result* c = new wg_result(*r);
  c->engine = nullptr;
  c->device = result_device(r);
  c->grid = result_grid(r);
  c->owned_bytes = std::max<uint64_t>(r->n * r->key_bytes, 256);
  if (hipSetDevice(c->device) != hipSuccess || hipMallocAsync(&c->owned, c->owned_bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return WG_ERR_OUT_OF_MEMORY;
  }
  // both runs, back to back
  const uint64_t na = r->n - r->n2;
  hipError_t err = wait_engine(r, s);
  if (na) err = hipMemcpyAsync(c->owned, r->keys, na * r->key_bytes, hipMemcpyDeviceToDevice, s);
  if (err == hipSuccess && r->n2)
    err = hipMemcpyAsync((uint8_t*)c->owned + na * r->key_bytes, r->keys2, r->n2 * r->key_bytes,
                         hipMemcpyDeviceToDevice, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (err != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFreeAsync(c->owned, s);
    delete c;
    return WG_ERR_DEVICE;
  }
  c->keys = c->owned;
  c->keys2 = r->n2 ? (const uint8_t*)c->owned + na * r->key_bytes : nullptr;
  c->release = std::move(release);
  if (bytes) *bytes = c->owned_bytes;
  *out = c;
  return WG_OK;
}

}  // namespace wg

// Helpers of the kernel-level entry points (single stages on caller arrays).
namespace {

// Shared prologue: options, stats, device and stream; the previous solve's queued work
// ordered before this call.
wg_status kernel_call_begin(wg_engine* e, const wg_options* opt_in, void* stream, wg_stats* st,
                            uint32_t key_bytes) {
  e->err.clear();
  wg_options o{};
  o.struct_size = sizeof(wg_options);
  if (opt_in) {
    if (opt_in->struct_size < 8 || opt_in->struct_size > sizeof(wg_options)) {
      e->err = "wg_options.struct_size is not a known size";
      return WG_ERR_INVALID_ARG;
    }
    std::memcpy(&o, opt_in, opt_in->struct_size);
  }
  if (key_bytes != 4 && key_bytes != 8) {
    e->err = "key_bytes must be 4 or 8";
    return WG_ERR_INVALID_ARG;
  }
  if (st) {
    uint64_t* ds = st->delta_sizes;
    uint64_t dc = st->delta_sizes_cap;
    std::memset(st, 0, sizeof(*st));
    st->delta_sizes = ds;
    st->delta_sizes_cap = dc;
    st->key_bytes = key_bytes;
  }
  e->timing = (o.flags & WG_STAGE_TIMING) != 0;
  e->timing_mask = 0xFFFFFFFFu;
  e->n_events = 0;
  return WG_OK;
}

template <typename K>
void sort_keys_impl(wg_engine* e, K* keys, K* tmp, uint64_t n, uint32_t key_bits, wg_stats* st) {
  const SortCfg c = e->tune[sizeof(K) == 8];
  const int passes = sort_passes((int)key_bits, c.rb);
  // the passes read their size from the control block and stop on none of its flags (the
  // block is written by a kernel whose argument carries it: a later call cannot overwrite a
  // host staging copy before this one's upload has run)
  Ctrl c0;
  std::memset(&c0, 0, sizeof(Ctrl));
  c0.m_in = n;
  launch_ctrl_set(e->stream, e->d_ctrl, c0);
  Bufs<K> b;
  std::memset(&b, 0, sizeof(b));
  b.cand[0] = keys;
  b.cand[1] = tmp;
  b.rcnt = e->d_rcnt;
  b.rtot = e->d_rtot;
  const uint64_t* n_ptr = &e->d_ctrl->m_in;
  for (int p = 0; p < passes; ++p) {
    launch_sort_pass<K>(e->stream, e->d_ctrl, n_ptr, c, b, p, false, stage(e, WG_STAGE_RADIX_HIST));
    launch_sort_pass<K>(e->stream, e->d_ctrl, n_ptr, c, b, p, true, stage(e, WG_STAGE_RADIX_PASS));
  }
  if (passes & 1)
    hip_check(e, hipMemcpyAsync(keys, tmp, n * sizeof(K), hipMemcpyDeviceToDevice, e->stream), "copy");
  if (st) {
    st->digit_bits = (uint32_t)c.rb;
    st->sort_passes = (uint32_t)passes;
    add_bytes(st, WG_STAGE_RADIX_HIST, (double)n * sizeof(K) * passes);
    add_bytes(st, WG_STAGE_RADIX_PASS, 2.0 * (double)n * sizeof(K) * passes);
  }
}

}  // namespace

extern "C" {

wg_status wg_engine_create(int device, wg_engine** out) { return wg_engine_create_ex(device, nullptr, out); }

wg_status wg_engine_create_ex(int device, const wg_allocator* allocator, wg_engine** out) {
  if (!out) return WG_ERR_INVALID_ARG;
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free)) return WG_ERR_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return WG_ERR_INVALID_ARG;
  wg_engine* e = new wg_engine();
  e->device = device;
  if (allocator) {
    e->alloc = *allocator;
    e->has_alloc = true;
  }
  try {
    hip_check(e, hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    hip_check(e, hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    const int cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    e->grid.stream = cu * 8;
    e->grid.scan = std::min(cu * 4, kScanBlocksMax);
    // defaults: 8-bit digits; the large tile for 32-bit keys, the small one for 64-bit keys
    // (measured best without tuning on R-MAT and SG workloads); wg_autotune refines them
    for (SortCfg& t : e->tune) {
      t.rb = 8;
      t.items = 16;
      t.blocks = std::min(cu * 4, kRadixBlocksMax);
    }
    e->tune[1].items = 8;
    // the fixed arrays come from the same allocator as the relation buffers, on the null
    // stream (e->stream is null until the first call)
    auto fixed = [&](void** p, size_t bytes) {
      *p = dev_alloc(e, bytes, nullptr);
      if (!*p) fail(e, WG_ERR_OUT_OF_MEMORY, "device allocation failed");
    };
    fixed((void**)&e->d_ctrl, kFixedBytes[0]);
    fixed((void**)&e->d_jtot, kFixedBytes[1]);
    fixed((void**)&e->d_bcnt, kFixedBytes[2]);
    fixed((void**)&e->d_rcnt, kFixedBytes[3]);
    fixed((void**)&e->d_rtot, kFixedBytes[4]);
    fixed((void**)&e->d_hits, sizeof(uint64_t) * e->grid.stream);
    fixed((void**)&e->d_bstart, kFixedBytes[5]);
    hip_check(e, hipHostMalloc((void**)&e->h_rb, 3 * sizeof(Readback)), "hipHostMalloc");
    hip_check(e, hipMemsetAsync(e->d_ctrl, 0, sizeof(Ctrl), nullptr), "hipMemsetAsync");
    for (int s = 0; s < 2; ++s)
      hip_check(e, hipEventCreateWithFlags(&e->ev_batch[s], hipEventDisableTiming), "hipEventCreate");
    hip_check(e, hipEventCreateWithFlags(&e->ev_done, hipEventDisableTiming), "hipEventCreate");
    hip_check(e, hipDeviceSynchronize(), "hipDeviceSynchronize");
  } catch (const Fail& f) {
    wg_engine_destroy(e);
    return f.st;
  }
  *out = e;
  return WG_OK;
}

void wg_engine_destroy(wg_engine* e) {
  if (!e) return;
  (void)hipSetDevice(e->device);
  (void)hipDeviceSynchronize();
  // everything is idle: the frees go on the null stream
  e->stream = nullptr;
  auto release = [&](DevBuf& b) {
    dev_free(e, b.p, b.bytes, nullptr);
    b.p = nullptr;
  };
  for (int s = 0; s < 2; ++s) {
    release(e->cand[s]);
    release(e->full[s]);
    release(e->fullB[s]);
    release(e->delta[s]);
  }
  release(e->E);
  release(e->U);
  release(e->R);
  release(e->Edst);
  release(e->rowa);
  release(e->rowb);
  release(e->off);
  release(e->rec);
  release(e->htab);
  release(e->tailrun);
  dev_free(e, e->d_ctrl, kFixedBytes[0], nullptr);
  dev_free(e, e->d_jtot, kFixedBytes[1], nullptr);
  dev_free(e, e->d_bcnt, kFixedBytes[2], nullptr);
  dev_free(e, e->d_rcnt, kFixedBytes[3], nullptr);
  dev_free(e, e->d_rtot, kFixedBytes[4], nullptr);
  dev_free(e, e->d_hits, sizeof(uint64_t) * e->grid.stream, nullptr);
  dev_free(e, e->d_bstart, kFixedBytes[5], nullptr);
  if (e->h_rb) (void)hipHostFree(e->h_rb);
  if (e->h_rec) (void)hipHostFree(e->h_rec);
  for (int s = 0; s < 2; ++s)
    if (e->ev_batch[s]) (void)hipEventDestroy(e->ev_batch[s]);
  if (e->ev_done) (void)hipEventDestroy(e->ev_done);
  for (hipEvent_t ev : e->events) (void)hipEventDestroy(ev);
  if (e->graph_exec) (void)hipGraphExecDestroy(e->graph_exec);
  if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
  (void)hipStreamSynchronize(nullptr);
  delete e;
}

wg_status wg_tc(wg_engine* e, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* o, void* stream, wg_result** out, wg_stats* st) {
  return solve(e, WG_QUERY_TC, 0, nullptr, d_src, d_dst, m, o, stream, out, st);
}

wg_status wg_sg(wg_engine* e, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* o, void* stream, wg_result** out, wg_stats* st) {
  return solve(e, WG_QUERY_SG, 0, nullptr, d_src, d_dst, m, o, stream, out, st);
}

wg_status wg_tc_batch(wg_engine* e, uint32_t num_instances, const uint64_t* d_offsets,
                      const uint32_t* d_src, const uint32_t* d_dst, uint64_t m, const wg_options* o,
                      void* stream, wg_result** out, wg_stats* st) {
  if (e && num_instances == 0) {
    e->err = "a batch needs at least one instance";
    return WG_ERR_INVALID_ARG;
  }
  return solve(e, WG_QUERY_TC, num_instances, d_offsets, d_src, d_dst, m, o, stream, out, st);
}

wg_status wg_sg_batch(wg_engine* e, uint32_t num_instances, const uint64_t* d_offsets,
                      const uint32_t* d_src, const uint32_t* d_dst, uint64_t m, const wg_options* o,
                      void* stream, wg_result** out, wg_stats* st) {
  if (e && num_instances == 0) {
    e->err = "a batch needs at least one instance";
    return WG_ERR_INVALID_ARG;
  }
  return solve(e, WG_QUERY_SG, num_instances, d_offsets, d_src, d_dst, m, o, stream, out, st);
}

wg_status wg_triangles(wg_engine* e, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                       const wg_options* o, void* stream, uint64_t* count_out, wg_stats* st) {
  if (!e) return WG_ERR_INVALID_ARG;
  if (!count_out) {
    e->err = "count_out is NULL";
    return WG_ERR_INVALID_ARG;
  }
  *count_out = 0;
  e->tri_count = 0;
  wg_result* res = nullptr;
  const wg_status r = solve(e, WG_QUERY_TRIANGLES, 0, nullptr, d_src, d_dst, m, o, stream, &res, st);
  wg_result_free(res);
  if (r == WG_OK) *count_out = e->tri_count;
  return r;
}

// ----- kernel-level entry points (single stages on caller arrays)

wg_status wg_sort_keys(wg_engine* e, void* d_keys, void* d_tmp, uint64_t n, uint32_t key_bytes,
                       uint32_t key_bits, const wg_options* o, void* stream, wg_stats* st) {
  if (!e) return WG_ERR_INVALID_ARG;
  const wg_status v = kernel_call_begin(e, o, stream, st, key_bytes);
  if (v != WG_OK) return v;
  if (n > 0 && (!d_keys || !d_tmp)) {
    e->err = "NULL key array with n > 0";
    return WG_ERR_INVALID_ARG;
  }
  if (key_bits == 0 || key_bits > 8 * key_bytes) {
    e->err = "key_bits must be 1..8*key_bytes";
    return WG_ERR_INVALID_ARG;
  }
  if (n > kMaxKeys) {
    e->err = "more than 2^32 - 16 keys";
    return WG_ERR_INVALID_ARG;
  }
  try {
    hip_check(e, hipSetDevice(e->device), "hipSetDevice");
    e->stream = (hipStream_t)stream;
    if (e->done_pending) hip_check(e, hipStreamWaitEvent(e->stream, e->ev_done, 0), "hipStreamWaitEvent");
    if (n > 1) {
      if (key_bytes == 4) sort_keys_impl<uint32_t>(e, (uint32_t*)d_keys, (uint32_t*)d_tmp, n, key_bits, st);
      else sort_keys_impl<uint64_t>(e, (uint64_t*)d_keys, (uint64_t*)d_tmp, n, key_bits, st);
    }
    hip_check(e, hipEventRecord(e->ev_done, e->stream), "hipEventRecord");
    e->done_pending = true;
    if (st) collect_timing(e, st);
    e->timing = false;
    return WG_OK;
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(e->stream);
    e->timing = false;
    return f.st;
  }
}

wg_status wg_merge_keys(wg_engine* e, const void* d_a, uint64_t na, const void* d_b, uint64_t nb, void* d_out,
                        uint32_t key_bytes, const wg_options* o, void* stream, wg_stats* st) {
  if (!e) return WG_ERR_INVALID_ARG;
  const wg_status v = kernel_call_begin(e, o, stream, st, key_bytes);
  if (v != WG_OK) return v;
  if ((na > 0 && !d_a) || (nb > 0 && !d_b) || (na + nb > 0 && !d_out)) {
    e->err = "NULL key array with a non-empty run";
    return WG_ERR_INVALID_ARG;
  }
  if (na > kMaxKeys || nb > kMaxKeys || na + nb > kMaxKeys) {
    e->err = "more than 2^32 - 16 keys";
    return WG_ERR_INVALID_ARG;
  }
  try {
    hip_check(e, hipSetDevice(e->device), "hipSetDevice");
    e->stream = (hipStream_t)stream;
    if (e->done_pending) hip_check(e, hipStreamWaitEvent(e->stream, e->ev_done, 0), "hipStreamWaitEvent");
    if (na + nb > 0) {
      const Ev ev = stage(e, WG_STAGE_MERGE);
      if (key_bytes == 4)
        launch_merge_pair<uint32_t>(e->stream, e->grid, (const uint32_t*)d_a, na, (const uint32_t*)d_b, nb,
                                    (uint32_t*)d_out, ev);
      else
        launch_merge_pair<uint64_t>(e->stream, e->grid, (const uint64_t*)d_a, na, (const uint64_t*)d_b, nb,
                                    (uint64_t*)d_out, ev);
      if (st) add_bytes(st, WG_STAGE_MERGE, 2.0 * (double)(na + nb) * key_bytes);
    }
    hip_check(e, hipEventRecord(e->ev_done, e->stream), "hipEventRecord");
    e->done_pending = true;
    if (st) collect_timing(e, st);
    e->timing = false;
    return WG_OK;
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(e->stream);
    e->timing = false;
    return f.st;
  }
}

uint32_t wg_result_instances(const wg_result* r) { return r ? r->num_inst : 0; }

wg_status wg_get_sort_config(const wg_engine* e, uint32_t key_bytes, wg_sort_config* out) {
  if (!e || !out || (key_bytes != 4 && key_bytes != 8)) return WG_ERR_INVALID_ARG;
  const SortCfg& c = e->tune[key_bytes == 8];
  out->digit_bits = (uint32_t)c.rb;
  out->tile_items = (uint32_t)(c.items == 8 ? 8 : (key_bytes == 4 ? 16 : 12));
  out->blocks = (uint32_t)c.blocks;
  out->reserved = 0;
  return WG_OK;
}

wg_status wg_set_sort_config(wg_engine* e, uint32_t key_bytes, const wg_sort_config* cfg) {
  if (!e) return WG_ERR_INVALID_ARG;
  if (!cfg || (key_bytes != 4 && key_bytes != 8) || cfg->digit_bits < (uint32_t)kRadixBitsMin ||
      cfg->digit_bits > (uint32_t)kRadixBitsMax ||
      (cfg->tile_items != 8 && cfg->tile_items != 12 && cfg->tile_items != 16) || cfg->blocks == 0 ||
      cfg->blocks > (uint32_t)kRadixBlocksMax) {
    e->err = "sort config: key_bytes 4 or 8, digit_bits 8..11, tile_items 8/12/16, blocks 1..2048";
    return WG_ERR_INVALID_ARG;
  }
  SortCfg& c = e->tune[key_bytes == 8];
  c.rb = (int)cfg->digit_bits;
  c.items = (int)cfg->tile_items;
  c.blocks = (int)cfg->blocks;
  return WG_OK;
}

wg_status wg_autotune(wg_engine* e, int query, uint32_t num_instances, const uint64_t* d_offsets,
                      const uint32_t* d_src, const uint32_t* d_dst, uint64_t m, const wg_options* opt_in,
                      uint32_t repeats, void* stream, wg_tune_report* rep) {
  if (!e) return WG_ERR_INVALID_ARG;
  if (query != WG_QUERY_TC && query != WG_QUERY_SG) {
    e->err = "query must be WG_QUERY_TC or WG_QUERY_SG";
    return WG_ERR_INVALID_ARG;
  }
  wg_options o{};
  o.struct_size = sizeof(wg_options);
  if (opt_in) {
    if (opt_in->struct_size < 8 || opt_in->struct_size > sizeof(wg_options)) {
      e->err = "wg_options.struct_size is not a known size";
      return WG_ERR_INVALID_ARG;
    }
    std::memcpy(&o, opt_in, opt_in->struct_size);
  }
  o.radix_digit_bits = 0;  // the trial configuration decides
  o.tile_items = 0;
  o.flags &= ~WG_STAGE_TIMING;
  if (repeats == 0) repeats = 2;
  // one untimed solve: allocations, the key type
  wg_stats st{};
  wg_result* res = nullptr;
  wg_status r = solve(e, query, num_instances, d_offsets, d_src, d_dst, m, &o, stream, &res, &st);
  wg_result_free(res);
  if (r != WG_OK) return r;
  const uint32_t kb = st.key_bytes ? st.key_bytes : 4;
  const SortCfg before = e->tune[kb == 8];
  int cu = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, e->device) == hipSuccess && prop.multiProcessorCount > 0)
    cu = prop.multiProcessorCount;
  std::vector<SortCfg> cands;
  for (int rb = kRadixBitsMin; rb <= kRadixBitsMax; ++rb)
    for (int items : {8, 16})
      for (int mult : {2, 4, 8}) {
        SortCfg c;
        c.rb = rb;
        c.items = items;
        c.blocks = std::min(cu * mult, kRadixBlocksMax);
        cands.push_back(c);
      }
  auto time_cfg = [&](const SortCfg& c, double& best) -> wg_status {
    best = 1e300;
    e->trial = &c;
    for (uint32_t i = 0; i <= repeats; ++i) {
      wg_stats s2{};
      wg_result* rr = nullptr;
      const wg_status q = solve(e, query, num_instances, d_offsets, d_src, d_dst, m, &o, stream, &rr, &s2);
      wg_result_free(rr);
      if (q != WG_OK) {
        e->trial = nullptr;
        return q;
      }
      if (i > 0) best = std::min(best, s2.solve_ms);  // the first run of a configuration warms it
    }
    e->trial = nullptr;
    return WG_OK;
  };
  double before_ms = 0;
  r = time_cfg(before, before_ms);
  if (r != WG_OK) return r;
  SortCfg best_cfg = before;
  double best_ms = before_ms;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->key_bytes = kb;
    rep->before_ms = before_ms;
  }
  for (const SortCfg& c : cands) {
    double ms = 0;
    r = time_cfg(c, ms);
    if (r != WG_OK) return r;
    if (rep && rep->trials < WG_TUNE_MAX_TRIALS) {
      wg_sort_config& t = rep->tried[rep->trials];
      t.digit_bits = (uint32_t)c.rb;
      t.tile_items = (uint32_t)(c.items == 8 ? 8 : (kb == 4 ? 16 : 12));
      t.blocks = (uint32_t)c.blocks;
      rep->tried_ms[rep->trials] = ms;
      rep->trials++;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best_cfg = c;
    }
  }
  e->tune[kb == 8] = best_cfg;
  if (rep) {
    rep->best.digit_bits = (uint32_t)best_cfg.rb;
    rep->best.tile_items = (uint32_t)(best_cfg.items == 8 ? 8 : (kb == 4 ? 16 : 12));
    rep->best.blocks = (uint32_t)best_cfg.blocks;
    rep->best_ms = best_ms;
  }
  return WG_OK;
}

wg_status wg_result_offsets(const wg_result* r, uint64_t* offsets_out, uint64_t capacity, void* stream) {
  const wg_status v = check_result(r);
  if (v != WG_OK) return v;
  if (!offsets_out || capacity < (uint64_t)r->num_inst + 1) {
    note(r, "offsets array missing or shorter than instances + 1");
    return WG_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  const uint64_t bytes = ((uint64_t)r->num_inst + 1) * 8;
  if (hipSetDevice(result_device(r)) != hipSuccess) return device_error(r, "hipSetDevice");
  const bool host = !is_device_pointer(offsets_out);
  uint64_t* dst = offsets_out;
  if (host && hipMallocAsync((void**)&dst, bytes, s) != hipSuccess) return device_error(r, "hipMallocAsync");
  const Grid g = result_grid(r);
  if (wait_engine(r, s) != hipSuccess) return device_error(r, "hipStreamWaitEvent");
  if (r->key_bytes == 4)
    launch_offsets<uint32_t>(s, g, (const uint32_t*)r->keys, r->n - r->n2, (const uint32_t*)r->keys2, r->n2,
                             2 * r->w, r->num_inst, dst);
  else
    launch_offsets<uint64_t>(s, g, (const uint64_t*)r->keys, r->n - r->n2, (const uint64_t*)r->keys2, r->n2,
                             2 * r->w, r->num_inst, dst);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = mark_engine_use(r, s);
  if (host) {
    if (err == hipSuccess) err = hipMemcpyAsync(offsets_out, dst, bytes, hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(dst, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
  }
  return err == hipSuccess ? WG_OK : device_error(r, "result offsets");
}

uint64_t wg_result_size(const wg_result* r) { return r ? r->n : 0; }

wg_status wg_result_copy(const wg_result* r, uint32_t* src_out, uint32_t* dst_out, uint64_t capacity,
                         void* stream) {
  const wg_status v = check_result(r);
  if (v != WG_OK) return v;
  if (r->n == 0) return WG_OK;
  if (!src_out || !dst_out || capacity < r->n) {
    note(r, "output arrays missing or too small");
    return WG_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(result_device(r)) != hipSuccess) return device_error(r, "hipSetDevice");
  const bool host = !is_device_pointer(src_out);
  const Grid g = result_grid(r);
  uint32_t* ds = src_out;
  uint32_t* dd = dst_out;
  uint32_t* tmp = nullptr;
  if (host) {
    if (hipMallocAsync((void**)&tmp, r->n * 8, s) != hipSuccess) return device_error(r, "hipMallocAsync");
    ds = tmp;
    dd = tmp + r->n;
  }
  if (wait_engine(r, s) != hipSuccess) return device_error(r, "hipStreamWaitEvent");
  if (r->key_bytes == 4)
    launch_unpack<uint32_t>(s, g, (const uint32_t*)r->keys, r->n - r->n2, (const uint32_t*)r->keys2, r->n2,
                            r->w, ds, dd);
  else
    launch_unpack<uint64_t>(s, g, (const uint64_t*)r->keys, r->n - r->n2, (const uint64_t*)r->keys2, r->n2,
                            r->w, ds, dd);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = mark_engine_use(r, s);
  if (host) {
    if (err == hipSuccess) err = hipMemcpyAsync(src_out, tmp, r->n * 4, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipMemcpyAsync(dst_out, tmp + r->n, r->n * 4, hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(tmp, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
  }
  return err == hipSuccess ? WG_OK : device_error(r, "result copy");
}

void wg_result_free(wg_result* r) {
  if (!r) return;
  if (r->owned) {
    // stream-ordered on the null stream, after every read enqueued on any stream (each
    // copy recorded an event), without waiting for the whole device
    (void)hipSetDevice(r->device);
    for (hipEvent_t ev : r->uses) (void)hipStreamWaitEvent(nullptr, ev, 0);
    (void)hipFreeAsync(r->owned, nullptr);
    if (r->release) r->release(r->owned_bytes);
  }
  for (hipEvent_t ev : r->uses) (void)hipEventDestroy(ev);
  delete r;
}


const char* wg_status_string(wg_status s) {
  switch (s) {
    case WG_OK: return "ok";
    case WG_ERR_INVALID_ARG: return "invalid argument";
    case WG_ERR_OUT_OF_MEMORY: return "out of device memory";
    case WG_ERR_CAPACITY: return "fixpoint exceeds the memory budget";
    case WG_ERR_DEVICE: return "device error";
    case WG_ERR_ITER_LIMIT: return "iteration limit reached";
    case WG_ERR_STALE: return "stale result";
    case WG_ERR_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* wg_last_error(const wg_engine* e) { return e ? e->err.c_str() : wg_call_error.c_str(); }

}  // extern "C"
