// Host side of the fixpoint engine: buffers, the prepare phase, the batched
// device-resident loop and the C ABI declared in include/wg.h.
//
// Engine rule (Section V): the host decides when the fixpoint terminates, the device
// decides every stage size.  The host enqueues K iterations at a time; each kernel
// reads its sizes from the device control block.  The host reads the control block
// back once per batch, after the next batch has already been enqueued (double-buffered
// submission, Section V-B), and adapts K by the paper's halving rule.

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wg.h"
#include "wg_launch.h"

using namespace wg;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

constexpr uint64_t kMaxKeys = 0xFFFFFFF0ull;        // offsets are 32-bit
constexpr uint64_t kEpochRefresh = 3'500'000ull;    // well below the 22-bit epoch range
constexpr uint32_t kMaxEvents = 1u << 16;

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct wg_engine {
  int device = 0;
  Grid grid{};
  Ctrl* d_ctrl = nullptr;
  Ctrl* h_up = nullptr;    // pinned upload staging
  Ctrl* h_down = nullptr;  // pinned readback, 2 slots
  hipEvent_t ev_batch[2] = {nullptr, nullptr};
  LbState* d_lb = nullptr;
  uint32_t* d_rcnt = nullptr;
  uint32_t* d_rtot = nullptr;
  DevBuf status[kLbCount];
  DevBuf cand[2], full[2], delta[2], E, U, R, Edst, rowa, rowb, off, hist;
  size_t allocated = 0;
  uint64_t budget = 0;
  uint64_t lb_launches = 0;
  uint64_t generation = 0;
  std::string err;
  // per-solve
  uint32_t key_bytes = 4;
  uint64_t cand_cap = 0, full_cap = 0, edge_cap = 0, row_cap = 0, dsz_cap = 0;
  uint64_t syncs = 0;
  // stage timing
  bool timing = false;
  uint32_t timing_mask = 0;
  std::vector<hipEvent_t> events;
  std::vector<int> event_kind;
  std::vector<int> event_launches;
  uint32_t n_events = 0;
  hipStream_t stream = nullptr;
  // result of the latest solve
  const void* res_keys = nullptr;
  uint64_t res_n = 0;
  int res_w = 16;
};

struct wg_result {
  wg_engine* engine;
  uint64_t generation;
  uint64_t n;
  int w;
  uint32_t key_bytes;
  const void* keys;
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

void free_buf(wg_engine* e, DevBuf& b) {
  if (b.p) {
    hip_check(e, hipFree(b.p), "hipFree");
    e->allocated -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

void alloc_buf(wg_engine* e, DevBuf& b, size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  if (e->budget && e->allocated + bytes > e->budget)
    fail(e, WG_ERR_CAPACITY, "device memory budget exceeded");
  void* p = nullptr;
  hipError_t r = hipMalloc(&p, bytes);
  if (r != hipSuccess) {
    (void)hipGetLastError();
    fail(e, WG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(r));
  }
  b.p = p;
  b.bytes = bytes;
  e->allocated += bytes;
}

// Ensure capacity without keeping contents.
void ensure(wg_engine* e, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return;
  free_buf(e, b);
  alloc_buf(e, b, bytes);
}

// Grow keeping the first `live` bytes (stream-ordered copy).
void grow_keep(wg_engine* e, DevBuf& b, size_t bytes, size_t live) {
  if (b.bytes >= bytes && b.p) return;
  DevBuf nb;
  alloc_buf(e, nb, bytes);
  if (live && b.p) hip_check(e, hipMemcpyAsync(nb.p, b.p, live, hipMemcpyDeviceToDevice, e->stream), "copy");
  hip_check(e, hipStreamSynchronize(e->stream), "sync");
  ++e->syncs;
  free_buf(e, b);
  b = nb;
}

void sync_stream(wg_engine* e) {
  hip_check(e, hipStreamSynchronize(e->stream), "hipStreamSynchronize");
  ++e->syncs;
}

uint64_t status_entries(int slot, uint64_t cand_cap, uint64_t full_cap, uint64_t edge_cap,
                        uint64_t row_cap, uint32_t key_bytes) {
  const uint32_t ptile = key_bytes == 4 ? pass_tile<uint32_t>() : pass_tile<uint64_t>();
  switch (slot) {
    case kLbJoin: return row_cap / kJoinTile + 2;
    case kLbPass: return (std::max(cand_cap, edge_cap) / ptile + 2) * kRadix;
    case kLbDedup: return std::max(cand_cap, edge_cap) / kDedupTile + 2;
    case kLbIndex: return edge_cap / kIndexTile + 2;
    case kLbFilter: return full_cap / kIndexTile + 2;
    default: return 0;
  }
}

// (Re)size every buffer for the current capacities.  `keep` preserves the live Full and
// delta contents described by the control block (grow-and-resume).
void size_buffers(wg_engine* e, bool keep, const Ctrl* c) {
  const uint64_t kb = e->key_bytes;
  for (int s = 0; s < 2; ++s) ensure(e, e->cand[s], e->cand_cap * kb);
  for (int s = 0; s < 2; ++s) {
    const bool live_f = keep && c && (uint32_t)s == c->full_side;
    const bool live_d = keep && c && (uint32_t)s == c->delta_side;
    if (live_f) grow_keep(e, e->full[s], e->full_cap * kb, c->F * kb);
    else ensure(e, e->full[s], e->full_cap * kb);
    if (live_d) grow_keep(e, e->delta[s], e->cand_cap * kb, c->D * kb);
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
  if (keep) grow_keep(e, e->hist, e->dsz_cap * 16, e->hist.bytes);
  else ensure(e, e->hist, e->dsz_cap * 16);
  for (int s = 0; s < kLbCount; ++s) {
    const uint64_t need = status_entries(s, e->cand_cap, e->full_cap, e->edge_cap, e->row_cap, e->key_bytes) * 8;
    if (need && (e->status[s].bytes < need || !e->status[s].p)) {
      ensure(e, e->status[s], need);
      // fresh memory must read as "not ready" for every epoch
      hip_check(e, hipMemsetAsync(e->status[s].p, 0, e->status[s].bytes, e->stream), "memset");
    }
  }
}

void refresh_epochs(wg_engine* e) {
  sync_stream(e);
  for (int s = 0; s < kLbCount; ++s)
    if (e->status[s].p) hip_check(e, hipMemsetAsync(e->status[s].p, 0, e->status[s].bytes, e->stream), "memset");
  hip_check(e, hipMemsetAsync(e->d_lb, 0, sizeof(LbState) * kLbCount, e->stream), "memset");
  e->lb_launches = 0;
}

template <typename K>
Bufs<K> make_bufs(wg_engine* e) {
  Bufs<K> b;
  for (int s = 0; s < 2; ++s) {
    b.cand[s] = (K*)e->cand[s].p;
    b.full[s] = (K*)e->full[s].p;
    b.delta[s] = (K*)e->delta[s].p;
  }
  b.E = (K*)e->E.p;
  b.U = (uint32_t*)e->U.p;
  b.R = (uint32_t*)e->R.p;
  b.Edst = (uint32_t*)e->Edst.p;
  b.rowa = (uint32_t*)e->rowa.p;
  b.rowb = (uint32_t*)e->rowb.p;
  b.off = (uint32_t*)e->off.p;
  b.hist = (uint64_t*)e->hist.p;
  b.lb = e->d_lb;
  for (int s = 0; s < kLbCount; ++s) b.status[s] = (uint64_t*)e->status[s].p;
  b.rcnt = e->d_rcnt;
  b.rtot = e->d_rtot;
  return b;
}

// ----- stage timing: events bracket every launch (begin, end) when WG_STAGE_TIMING is set.
hipEvent_t next_event(wg_engine* e) {
  if (e->n_events >= e->events.size()) {
    hipEvent_t ev;
    hip_check(e, hipEventCreate(&ev), "hipEventCreate");
    e->events.push_back(ev);
    e->event_kind.push_back(-1);
    e->event_launches.push_back(1);
  }
  return e->events[e->n_events];
}

void begin(wg_engine* e, int kind) {
  if (!e->timing || !((e->timing_mask >> kind) & 1u) || e->n_events + 2 > kMaxEvents) return;
  hip_check(e, hipEventRecord(next_event(e), e->stream), "hipEventRecord");
  e->event_kind[e->n_events] = -1;
  ++e->n_events;
}

void end(wg_engine* e, int kind, int launches = 1) {
  if (!e->timing || e->n_events == 0 || e->event_kind[e->n_events - 1] != -1) return;
  hip_check(e, hipEventRecord(next_event(e), e->stream), "hipEventRecord");
  e->event_kind[e->n_events] = kind;
  e->event_launches[e->n_events] = launches;
  ++e->n_events;
}

void collect_timing(wg_engine* e, wg_stats* st) {
  if (!e->timing || e->n_events < 2) return;
  hip_check(e, hipEventSynchronize(e->events[e->n_events - 1]), "hipEventSynchronize");
  for (uint32_t i = 1; i < e->n_events; ++i) {
    const int k = e->event_kind[i];
    if (k < 0 || e->event_kind[i - 1] != -1) continue;
    float ms = 0.f;
    hip_check(e, hipEventElapsedTime(&ms, e->events[i - 1], e->events[i]), "hipEventElapsedTime");
    st->stage_ms[k] += ms;
    st->stage_launches[k] += (uint64_t)e->event_launches[i];
  }
}

// ----- pipeline pieces
template <typename K>
void enqueue_sort(wg_engine* e, const Bufs<K>& b, const uint64_t* n_ptr, int passes) {
  // one event pair brackets all passes, so stage_ms / launches is the mean pass time
  begin(e, WG_STAGE_RADIX_PASS);
  for (int p = 0; p < passes; ++p)
    launch_radix_pass<K>(e->stream, e->grid, e->d_ctrl, n_ptr, b.cand[p & 1], b.cand[(p + 1) & 1], p, b);
  end(e, WG_STAGE_RADIX_PASS, passes);
  e->lb_launches += passes;
}

template <typename K>
void enqueue_iteration(wg_engine* e, const Bufs<K>& b, int kind, int w, int passes) {
  begin(e, WG_STAGE_JOIN_COUNT);
  launch_join_count<K>(e->stream, e->grid, kind, e->d_ctrl, b, w);
  end(e, WG_STAGE_JOIN_COUNT);
  begin(e, WG_STAGE_JOIN_EMIT);
  launch_join_emit<K>(e->stream, e->grid, kind, e->d_ctrl, b, w);
  end(e, WG_STAGE_JOIN_EMIT);
  enqueue_sort<K>(e, b, &e->d_ctrl->C, passes);
  begin(e, WG_STAGE_DEDUP_DIFF);
  launch_dedup_diff<K>(e->stream, e->grid, kModeIter, e->d_ctrl, &e->d_ctrl->C, b.cand[passes & 1], b);
  end(e, WG_STAGE_DEDUP_DIFF);
  begin(e, WG_STAGE_MERGE);
  launch_merge<K>(e->stream, e->grid, e->d_ctrl, b);
  end(e, WG_STAGE_MERGE);
  e->lb_launches += 3;
}

void read_ctrl(wg_engine* e, int slot) {
  hip_check(e, hipMemcpyAsync(&e->h_down[slot], e->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, e->stream),
            "readback");
  hip_check(e, hipEventRecord(e->ev_batch[slot], e->stream), "hipEventRecord");
}

Ctrl wait_ctrl(wg_engine* e, int slot) {
  hip_check(e, hipEventSynchronize(e->ev_batch[slot]), "hipEventSynchronize");
  ++e->syncs;
  return e->h_down[slot];
}

// Grow the buffers after an overflow and clear the flag; the loop then resumes from the
// last completed iteration, whose Full and delta are intact.
void grow_and_resume(wg_engine* e, const Ctrl& c, bool hooked) {
  uint64_t cand = e->cand_cap, full = e->full_cap, dsz = e->dsz_cap;
  bool clear_hook = false;
  if (c.overflow & 1u) {
    if (hooked && c.C <= e->cand_cap) clear_hook = true;  // forced by the test hook
    else cand = std::max(cand * 2, c.C + c.C / 4);
  }
  if (c.overflow & 4u) cand = std::max(cand * 2, c.N + c.N / 4);
  if (c.overflow & 2u) full = std::max(full * 2, (c.F + c.N) + (c.F + c.N) / 4);
  if (c.overflow & 8u) dsz = dsz * 2;
  if (cand > kMaxKeys || full > kMaxKeys)
    fail(e, WG_ERR_CAPACITY, "relation exceeds 2^32 keys per buffer");
  e->cand_cap = cand;
  e->full_cap = full;
  e->dsz_cap = dsz;
  size_buffers(e, true, &c);
  launch_resume(e->stream, e->d_ctrl, e->cand_cap, e->full_cap, e->dsz_cap, clear_hook ? 1u : 0u);
}

int field_bits(uint32_t maxid) {
  if (maxid < (1u << 16)) return 16;
  if (maxid < (1u << 24)) return 24;
  return 32;
}

void add_bytes(wg_stats* st, int k, double b) { st->stage_bytes[k] += (uint64_t)b; }

// Algorithmic HBM bytes per kernel kind (what each stage must stream at minimum).
void bytes_model(wg_stats* st, int query, uint32_t kb, int passes, uint64_t m,
                 const std::vector<uint64_t>& N, const std::vector<uint64_t>& C, uint64_t base_cand) {
  // prepare: max scan + pack + sort + dedup of m edges + index
  add_bytes(st, WG_STAGE_PREPARE, 8.0 * m + (8.0 + kb) * m + (kb + 12.0) * m);
  add_bytes(st, WG_STAGE_RADIX_PASS, 3.0 * kb * m * passes);
  add_bytes(st, WG_STAGE_DEDUP_DIFF, (double)kb * m + (double)kb * N[0] * (query == WG_QUERY_TC ? 3 : 0));
  if (query == WG_QUERY_SG) {
    add_bytes(st, WG_STAGE_JOIN_EMIT, (double)(kb + 8) * base_cand);
    add_bytes(st, WG_STAGE_RADIX_PASS, 3.0 * kb * base_cand * passes);
    add_bytes(st, WG_STAGE_DEDUP_DIFF, (double)kb * base_cand + 2.0 * kb * N[0]);
  }
  uint64_t F = N[0];
  const double row_bytes = query == WG_QUERY_TC ? 8.0 : 12.0;
  const double edst = query == WG_QUERY_TC ? 4.0 : 8.0;
  for (size_t i = 1; i < N.size(); ++i) {
    const double D = (double)N[i - 1], c = (double)C[i], n = (double)N[i];
    add_bytes(st, WG_STAGE_JOIN_COUNT, D * (kb + row_bytes));
    add_bytes(st, WG_STAGE_JOIN_EMIT, D * (kb + row_bytes) + c * (edst + kb));
    add_bytes(st, WG_STAGE_RADIX_PASS, 3.0 * c * kb * passes);
    add_bytes(st, WG_STAGE_DEDUP_DIFF, (c + n) * kb);
    if (N[i] > 0) add_bytes(st, WG_STAGE_MERGE, 2.0 * ((double)F + n) * kb);
    F += N[i];
  }
}

template <typename K>
wg_status run(wg_engine* e, int query, const uint32_t* src, const uint32_t* dst, uint64_t m,
              const wg_options& o, int w, wg_stats* st) {
  const int key_bits = 2 * w;
  const int passes = (key_bits + kRadixBits - 1) / kRadixBits;
  e->key_bytes = sizeof(K);
  e->edge_cap = std::max<uint64_t>(e->edge_cap, m);
  e->cand_cap = std::max<uint64_t>({e->cand_cap, 2 * m, 1u << 20});
  e->full_cap = std::max<uint64_t>({e->full_cap, 2 * m, 1u << 20});
  e->cand_cap = std::min(e->cand_cap, kMaxKeys);
  e->full_cap = std::min(e->full_cap, kMaxKeys);
  e->dsz_cap = std::max<uint64_t>(e->dsz_cap, 4096);
  size_buffers(e, false, nullptr);
  if (e->lb_launches > kEpochRefresh) refresh_epochs(e);

  Ctrl& c0 = *e->h_up;
  std::memset(&c0, 0, sizeof(Ctrl));
  c0.m_in = m;
  c0.cand_cap = e->cand_cap;
  c0.delta_cap = e->cand_cap;
  c0.full_cap = e->full_cap;
  c0.dsz_cap = e->dsz_cap;
  c0.max_iter = (uint32_t)std::min<uint64_t>(o.max_iterations, 0xFFFFFFFFu);
  c0.force_overflow_at = (uint32_t)std::min<uint64_t>(o.force_overflow_at_iter, 0xFFFFFFFFu);
  hip_check(e, hipMemcpyAsync(e->d_ctrl, e->h_up, sizeof(Ctrl), hipMemcpyHostToDevice, e->stream), "upload");

  // ---- prepare: sort + dedup E, edge index, seed (Section IV-A: E sorted once)
  Bufs<K> b = make_bufs<K>(e);
  begin(e, WG_STAGE_PREPARE);
  launch_pack<K>(e->stream, e->grid, src, dst, m, w, b.cand[0]);
  end(e, WG_STAGE_PREPARE);
  enqueue_sort<K>(e, b, &e->d_ctrl->m_in, passes);
  const int mode = query == WG_QUERY_TC ? (kModeEdges | kModeSeed) : kModeEdges;
  begin(e, WG_STAGE_DEDUP_DIFF);
  launch_dedup_diff<K>(e->stream, e->grid, mode, e->d_ctrl, &e->d_ctrl->m_in, b.cand[passes & 1], b);
  end(e, WG_STAGE_DEDUP_DIFF);
  begin(e, WG_STAGE_PREPARE);
  launch_edge_index<K>(e->stream, e->grid, e->d_ctrl, b, w);
  end(e, WG_STAGE_PREPARE);
  e->lb_launches += 2;

  uint64_t base_cand = 0;
  if (query == WG_QUERY_SG) {
    // base rule: Delta^0 = Full = {(x, y) : E(p, x), E(p, y), x != y}, sorted + deduplicated
    for (;;) {
      b = make_bufs<K>(e);
      begin(e, WG_STAGE_JOIN_COUNT);
      launch_join_count<K>(e->stream, e->grid, kJoinSGBase, e->d_ctrl, b, w);
      end(e, WG_STAGE_JOIN_COUNT);
      begin(e, WG_STAGE_JOIN_EMIT);
      launch_join_emit<K>(e->stream, e->grid, kJoinSGBase, e->d_ctrl, b, w);
      end(e, WG_STAGE_JOIN_EMIT);
      enqueue_sort<K>(e, b, &e->d_ctrl->C, passes);
      begin(e, WG_STAGE_DEDUP_DIFF);
      launch_dedup_diff<K>(e->stream, e->grid, kModeSeed, e->d_ctrl, &e->d_ctrl->C, b.cand[passes & 1], b);
      end(e, WG_STAGE_DEDUP_DIFF);
      e->lb_launches += 2;
      read_ctrl(e, 0);
      const Ctrl c = wait_ctrl(e, 0);
      if (c.error) fail(e, WG_ERR_DEVICE, "device wait expired in the base stage");
      if (!c.overflow) {
        base_cand = c.C;
        break;
      }
      grow_and_resume(e, c, false);
      if (st) st->resumes++;
    }
  }

  // ---- the semi-naive loop, K iterations per host check
  const int kind = query == WG_QUERY_TC ? kJoinTC : kJoinSG;
  uint32_t K_batch = o.batch_k ? o.batch_k : (query == WG_QUERY_TC ? 30u : 10u);
  const bool adaptive = (o.batch_k == 0 && query == WG_QUERY_TC);
  if (o.loop_mode == WG_LOOP_HOST) K_batch = 1;
  const bool hooked = o.force_overflow_at_iter != 0;
  Ctrl c{};
  int slot = 0;
  uint64_t prev_D = 0;
  bool have_prev = false;
  auto enqueue_iters = [&](uint32_t k) {
    b = make_bufs<K>(e);
    for (uint32_t i = 0; i < k; ++i) enqueue_iteration<K>(e, b, kind, w, passes);
  };
  auto enqueue_batch = [&](uint32_t k, int sl) {
    enqueue_iters(k);
    read_ctrl(e, sl);
  };
  const uint64_t per_iter_launches = 3 + (uint64_t)passes;
  constexpr uint32_t kSpec = 4;
  enqueue_batch(K_batch, slot);
  for (;;) {
    // While the host waits on this batch, the device runs a short speculative batch
    // behind it (Section V-B overlaps the next batch with the host check); after the
    // fixpoint its launches are no-ops, so it is kept short.
    const uint32_t spec = std::min(K_batch, kSpec);
    const bool speculate = e->lb_launches + per_iter_launches * (K_batch + spec) < kEpochRefresh;
    if (speculate) enqueue_iters(spec);
    c = wait_ctrl(e, slot);
    if (c.error | c.overflow | c.done | c.limit_hit) sync_stream(e);
    if (c.error) fail(e, WG_ERR_DEVICE, "device wait expired (lookback spin limit)");
    if (c.overflow) {
      grow_and_resume(e, c, hooked);
      if (st) st->resumes++;
      if (e->lb_launches > kEpochRefresh) refresh_epochs(e);
      enqueue_batch(K_batch, slot);
      continue;
    }
    if (c.done || c.limit_hit) break;
    if (adaptive) {
      // Section V-B: halve K when the batch's last/first delta-size ratio is below 0.1
      const uint64_t first = have_prev ? prev_D : c.D0;
      if (first > 0 && (double)c.D / (double)first < 0.1) K_batch = std::max(1u, K_batch / 2);
    }
    prev_D = c.D;
    have_prev = true;
    if (!speculate) refresh_epochs(e);
    slot ^= 1;
    enqueue_batch(K_batch, slot);
  }
  if (c.limit_hit && !c.done) fail(e, WG_ERR_ITER_LIMIT, "max_iterations reached before the fixpoint");

  b = make_bufs<K>(e);
  if (query == WG_QUERY_SG && (o.flags & WG_SG_IRREFLEXIVE)) {
    begin(e, WG_STAGE_PREPARE);
    launch_filter_offdiag<K>(e->stream, e->grid, e->d_ctrl, b, w);
    end(e, WG_STAGE_PREPARE);
    e->lb_launches += 1;
    read_ctrl(e, 0);
    c = wait_ctrl(e, 0);
    if (c.error) fail(e, WG_ERR_DEVICE, "device wait expired in the diagonal filter");
  }
  e->res_keys = b.full[c.full_side];
  e->res_n = c.F;
  e->res_w = w;

  if (st) {
    st->iterations = c.iter;
    st->result_tuples = c.F;
    st->base_tuples = c.D0;
    st->join_candidates = c.total_cand;
    st->field_bits = (uint32_t)w;
    st->key_bytes = (uint32_t)sizeof(K);
    std::vector<uint64_t> h(2 * ((size_t)c.iter + 1));
    hip_check(e, hipMemcpy(h.data(), e->hist.p, h.size() * 8, hipMemcpyDeviceToHost), "hist readback");
    ++e->syncs;
    std::vector<uint64_t> N(c.iter + 1), C(c.iter + 1);
    for (size_t i = 0; i <= c.iter; ++i) {
      N[i] = h[2 * i];
      C[i] = h[2 * i + 1];
    }
    if (st->delta_sizes)
      for (uint64_t i = 0; i < std::min<uint64_t>(st->delta_sizes_cap, N.size()); ++i) st->delta_sizes[i] = N[i];
    bytes_model(st, query, sizeof(K), passes, m, N, C, base_cand);
    collect_timing(e, st);
  }
  return WG_OK;
}

wg_status solve(wg_engine* e, int query, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
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
  if (m >= kMaxKeys / 2) {
    e->err = "too many edges";
    return WG_ERR_INVALID_ARG;
  }
  if (o.radix_field_bits != 0 && o.radix_field_bits != 16 && o.radix_field_bits != 24 &&
      o.radix_field_bits != 32) {
    e->err = "radix_field_bits must be 0, 16, 24 or 32";
    return WG_ERR_INVALID_ARG;
  }
  if (o.loop_mode > WG_LOOP_HOST || (o.flags & ~(WG_SG_IRREFLEXIVE | WG_STAGE_TIMING))) {
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
    e->generation++;
    e->res_keys = nullptr;
    e->res_n = 0;
    e->syncs = 0;
    e->budget = o.mem_budget_bytes;
    e->timing = (o.flags & WG_STAGE_TIMING) != 0;
    e->timing_mask = o.timing_stages ? o.timing_stages : 0xFFFFFFFFu;
    e->n_events = 0;
    if (m == 0) {
      if (st && st->delta_sizes && st->delta_sizes_cap) st->delta_sizes[0] = 0;
    } else {
      // largest id -> radix field width (Section V-C); the one synchronisation before the loop
      std::memset(e->h_up, 0, sizeof(Ctrl));
      hip_check(e, hipMemcpyAsync(e->d_ctrl, e->h_up, sizeof(Ctrl), hipMemcpyHostToDevice, e->stream), "upload");
      launch_max_id(e->stream, e->grid, e->d_ctrl, d_src, d_dst, m);
      read_ctrl(e, 0);
      const Ctrl c = wait_ctrl(e, 0);
      int w = field_bits(c.maxid);
      if (o.radix_field_bits) {
        if ((int)o.radix_field_bits < w) {
          e->err = "radix_field_bits does not cover the largest vertex id";
          return WG_ERR_INVALID_ARG;
        }
        w = (int)o.radix_field_bits;
      }
      wg_status r = (2 * w <= 32) ? run<uint32_t>(e, query, d_src, d_dst, m, o, w, st)
                                  : run<uint64_t>(e, query, d_src, d_dst, m, o, w, st);
      if (r != WG_OK) return r;
    }
    wg_result* res = new wg_result{e, e->generation, e->res_n, e->res_w, e->key_bytes, e->res_keys};
    *out = res;
    if (st) {
      st->host_syncs = e->syncs;
      st->solve_ms = now_ms() - t0;
    }
    return WG_OK;
  } catch (const Fail& f) {
    if (f.st != WG_ERR_DEVICE) {
      (void)hipStreamSynchronize(e->stream);
      // capacity errors leave device-side flags set; the next solve re-uploads the block
    }
    return f.st;
  }
}

}  // namespace

extern "C" {

wg_status wg_engine_create(int device, wg_engine** out) {
  if (!out) return WG_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return WG_ERR_INVALID_ARG;
  wg_engine* e = new wg_engine();
  e->device = device;
  try {
    hip_check(e, hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    hip_check(e, hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    const int cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    e->grid.persistent = cu * 4;
    e->grid.stream = cu * 8;
    e->grid.sort = std::min(cu * 4, kSortBlocksMax);
    hip_check(e, hipMalloc((void**)&e->d_ctrl, sizeof(Ctrl)), "hipMalloc");
    hip_check(e, hipHostMalloc((void**)&e->h_up, sizeof(Ctrl)), "hipHostMalloc");
    hip_check(e, hipHostMalloc((void**)&e->h_down, 2 * sizeof(Ctrl)), "hipHostMalloc");
    hip_check(e, hipMalloc((void**)&e->d_lb, sizeof(LbState) * kLbCount), "hipMalloc");
    hip_check(e, hipMalloc((void**)&e->d_rcnt, sizeof(uint32_t) * kRadix * kSortBlocksMax), "hipMalloc");
    hip_check(e, hipMalloc((void**)&e->d_rtot, sizeof(uint32_t) * kRadix), "hipMalloc");
    hip_check(e, hipMemset(e->d_lb, 0, sizeof(LbState) * kLbCount), "hipMemset");
    hip_check(e, hipMemset(e->d_ctrl, 0, sizeof(Ctrl)), "hipMemset");
    for (int s = 0; s < 2; ++s)
      hip_check(e, hipEventCreateWithFlags(&e->ev_batch[s], hipEventDisableTiming), "hipEventCreate");
    hip_check(e, hipDeviceSynchronize(), "hipDeviceSynchronize");
  } catch (const Fail&) {
    wg_engine_destroy(e);
    return WG_ERR_DEVICE;
  }
  *out = e;
  return WG_OK;
}

void wg_engine_destroy(wg_engine* e) {
  if (!e) return;
  (void)hipSetDevice(e->device);
  (void)hipDeviceSynchronize();
  auto release = [&](DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
  };
  for (int s = 0; s < 2; ++s) {
    release(e->cand[s]);
    release(e->full[s]);
    release(e->delta[s]);
  }
  release(e->E);
  release(e->U);
  release(e->R);
  release(e->Edst);
  release(e->rowa);
  release(e->rowb);
  release(e->off);
  release(e->hist);
  for (int s = 0; s < kLbCount; ++s) release(e->status[s]);
  if (e->d_ctrl) (void)hipFree(e->d_ctrl);
  if (e->d_lb) (void)hipFree(e->d_lb);
  if (e->d_rcnt) (void)hipFree(e->d_rcnt);
  if (e->d_rtot) (void)hipFree(e->d_rtot);
  if (e->h_up) (void)hipHostFree(e->h_up);
  if (e->h_down) (void)hipHostFree(e->h_down);
  for (int s = 0; s < 2; ++s)
    if (e->ev_batch[s]) (void)hipEventDestroy(e->ev_batch[s]);
  for (hipEvent_t ev : e->events) (void)hipEventDestroy(ev);
  delete e;
}

wg_status wg_tc(wg_engine* e, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* o, void* stream, wg_result** out, wg_stats* st) {
  return solve(e, WG_QUERY_TC, d_src, d_dst, m, o, stream, out, st);
}

wg_status wg_sg(wg_engine* e, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* o, void* stream, wg_result** out, wg_stats* st) {
  return solve(e, WG_QUERY_SG, d_src, d_dst, m, o, stream, out, st);
}

uint64_t wg_result_size(const wg_result* r) { return r ? r->n : 0; }

wg_status wg_result_copy(const wg_result* r, uint32_t* src_out, uint32_t* dst_out, uint64_t capacity,
                         void* stream) {
  if (!r || !r->engine) return WG_ERR_INVALID_ARG;
  wg_engine* e = r->engine;
  if (r->generation != e->generation) {
    e->err = "result is stale: the engine ran another solve";
    return WG_ERR_STALE;
  }
  if (r->n == 0) return WG_OK;
  if (!src_out || !dst_out || capacity < r->n) {
    e->err = "output arrays missing or too small";
    return WG_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    hip_check(e, hipSetDevice(e->device), "hipSetDevice");
    hipPointerAttribute_t a{};
    bool host = false;
    if (hipPointerGetAttributes(&a, src_out) != hipSuccess) {
      (void)hipGetLastError();
      host = true;
    } else {
      host = a.type != hipMemoryTypeDevice;
    }
    Grid g = e->grid;
    if (!host) {
      if (r->key_bytes == 4)
        launch_unpack<uint32_t>(s, g, (const uint32_t*)r->keys, r->n, r->w, src_out, dst_out);
      else
        launch_unpack<uint64_t>(s, g, (const uint64_t*)r->keys, r->n, r->w, src_out, dst_out);
      hip_check(e, hipGetLastError(), "unpack launch");
      return WG_OK;
    }
    uint32_t* tmp = nullptr;
    hip_check(e, hipMalloc((void**)&tmp, r->n * 8), "hipMalloc");
    if (r->key_bytes == 4)
      launch_unpack<uint32_t>(s, g, (const uint32_t*)r->keys, r->n, r->w, tmp, tmp + r->n);
    else
      launch_unpack<uint64_t>(s, g, (const uint64_t*)r->keys, r->n, r->w, tmp, tmp + r->n);
    hipError_t e1 = hipMemcpyAsync(src_out, tmp, r->n * 4, hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipMemcpyAsync(dst_out, tmp + r->n, r->n * 4, hipMemcpyDeviceToHost, s);
    hipError_t e3 = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    hip_check(e, e1, "copy");
    hip_check(e, e2, "copy");
    hip_check(e, e3, "sync");
    return WG_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

void wg_result_free(wg_result* r) { delete r; }

const char* wg_status_string(wg_status s) {
  switch (s) {
    case WG_OK: return "ok";
    case WG_ERR_INVALID_ARG: return "invalid argument";
    case WG_ERR_OUT_OF_MEMORY: return "out of device memory";
    case WG_ERR_CAPACITY: return "fixpoint exceeds the memory budget";
    case WG_ERR_DEVICE: return "device error";
    case WG_ERR_ITER_LIMIT: return "iteration limit reached";
    case WG_ERR_STALE: return "stale result";
  }
  return "unknown status";
}

const char* wg_last_error(const wg_engine* e) { return e ? e->err.c_str() : ""; }

}  // extern "C"
