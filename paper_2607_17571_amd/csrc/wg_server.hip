// Request server: continuous batching of TC / SG solves on one device.
//
// Each slot is a worker thread with its own engine and HIP stream, so the solves of
// different slots overlap on the device.  Requests wait in a queue and are admitted to
// a free slot as soon as the device-memory budget allows: a request reserves an
// estimate of its peak memory (bytes per edge, learned per query kind from completed
// solves), and the reservations of running solves, the resident buffers of idle
// engines, resident results and queued inputs together stay within the budget.
// A solve that outgrows its reservation asks the server for more (it waits while other
// solves still hold the memory); if every running solve is waiting, the youngest gives
// up, frees its memory and is queued again with a larger reservation -- with the whole
// budget if need be, in which case it runs alone.  Results stay resident on the device
// until the client frees them.
//
// Serving is an addition to the paper's method (which evaluates one query at a time);
// every solve runs the same engine as wg_tc / wg_sg, so a result is the same alone and
// in any mix.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/wg.h"
#include "wg_internal.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum JobPhase : int { kQueued = 0, kRunning = 1, kDone = 2 };

constexpr uint64_t kMinReservation = 64ull << 20;
constexpr uint32_t kMaxPassOver = 16;  // later requests may pass a waiting one this often
constexpr uint64_t kHoldCandidates = 1ull << 21;  // an iteration this large marks a long solve
constexpr double kMaxMemoryWaitMs = 5000.0;  // a growing solve waits this long for memory

struct JobState {
  int query = 0;
  wg_options opts{};
  uint32_t* d_edges = nullptr;  // src (m) then dst (m), owned by the server
  uint64_t m = 0;
  uint64_t input_bytes = 0;
  uint64_t reservation = 0;
  bool exclusive = false;  // needs the whole budget: blocks later requests until it runs
  uint32_t requeues = 0;
  uint32_t passed_over = 0;
  int phase = kQueued;
  bool abandoned = false;  // the client freed its handle before the job finished
  std::atomic<bool> cancel{false};
  wg_status status = WG_OK;
  wg_result* result = nullptr;
  bool result_taken = false;
  wg_stats stats{};
  std::vector<uint64_t> deltas;
  std::string error;
  double t_submit = 0, t_start = 0, t_end = 0;
  uint64_t peak_bytes = 0;
};

// State shared with result and job handles, which may outlive the server.
struct Core {
  std::mutex mu;
  std::condition_variable cv;
  int64_t held = 0;    // resident results + queued inputs (bytes)
  bool alive = true;   // false once wg_server_destroy has finished every job
  double t0 = 0;       // server clock origin
};

struct Slot {
  wg_engine* engine = nullptr;
  hipStream_t stream = nullptr;
  std::thread thread;
  std::shared_ptr<JobState> job;  // running job
  uint64_t reservation = 0;       // budget granted to the running job
  uint64_t resident = 0;          // engine buffers kept between jobs
  bool waiting_memory = false;
  bool trim_requested = false;
  double busy_since = 0;
};

}  // namespace

struct wg_server {
  int device = 0;
  uint64_t budget = 0;
  hipStream_t copy_stream = nullptr;  // input staging (stream-ordered allocations)
  std::vector<std::unique_ptr<Slot>> slots;
  std::shared_ptr<Core> core;
  std::deque<std::shared_ptr<JobState>> queue;
  double alpha[2] = {8192.0, 8192.0};  // reservation bytes per edge (TC, SG)
  bool stop = false;
  double t0 = 0;
  double hold_after_ms = 8.0;  // a solve running longer holds back admissions (< 0: never)
  wg_server_stats st{};
  std::string err;
};

// A job handle keeps the shared state alive; it reaches the server itself only while
// core->alive (after wg_server_destroy every job is done and needs nothing of the server).
struct wg_job {
  wg_server* server;
  std::shared_ptr<Core> core;
  std::shared_ptr<JobState> s;
};

namespace {

// Memory in use outside slot `i` (caller holds the lock).
uint64_t usage_except(const wg_server* sv, size_t i) {
  uint64_t u = (uint64_t)std::max<int64_t>(sv->core->held, 0);
  for (size_t k = 0; k < sv->slots.size(); ++k) {
    if (k == i) continue;
    const Slot& s = *sv->slots[k];
    u += s.job ? std::max(s.reservation, s.resident) : s.resident;
  }
  return u;
}

// Ask idle slots holding buffers to free them (caller holds the lock).
bool request_trims(wg_server* sv, size_t except) {
  bool any = false;
  for (size_t k = 0; k < sv->slots.size(); ++k) {
    Slot& s = *sv->slots[k];
    if (k != except && !s.job && s.resident > 0 && !s.trim_requested) {
      s.trim_requested = true;
      any = true;
    }
  }
  if (any) sv->core->cv.notify_all();
  return any;
}

// Starting reservation: the learned bytes per edge times m, at most one slot's share of
// the budget (a solve that needs more grows through the grow hook).
uint64_t estimate(const wg_server* sv, const JobState& j) {
  const double est = sv->alpha[j.query == WG_QUERY_SG] * (double)j.m;
  const uint64_t share = std::max<uint64_t>(kMinReservation, sv->budget / sv->slots.size());
  return std::min<uint64_t>(share, std::max<uint64_t>(kMinReservation, (uint64_t)est));
}

// Next admissible request for slot i, or null (caller holds the lock).  Its reservation
// is returned in *grant.
std::shared_ptr<JobState> pick(wg_server* sv, size_t i, uint64_t* grant) {
  Slot& me = *sv->slots[i];
  bool others_run = false;
  const double now = now_ms();
  for (size_t k = 0; k < sv->slots.size(); ++k) {
    const Slot& o = *sv->slots[k];
    if (k == i || !o.job) continue;
    others_run = true;
    if (o.waiting_memory) return nullptr;  // memory that frees up goes to waiting solves first
    // a long solve (the heavy tail of the mix) finishes faster alone than beside new
    // arrivals; those wait until it ends (its slot notifies at the end).  A solve is long
    // once it has run hold_after, or as soon as one of its host checks has read back an
    // iteration of kHoldCandidates candidates or more (a large fixpoint, known a few
    // milliseconds before the clock would tell)
    if (sv->hold_after_ms >= 0 &&
        (now - o.busy_since > sv->hold_after_ms || wg::engine_seen_candidates(o.engine) >= kHoldCandidates))
      return nullptr;
  }
  const uint64_t others = usage_except(sv, i);
  const uint64_t held = (uint64_t)std::max<int64_t>(sv->core->held, 0);
  for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
    JobState& j = **it;
    // a reservation that cannot fit beside the held results and inputs needs the device alone
    if (!j.exclusive && j.reservation + held > sv->budget) j.exclusive = true;
    if (j.exclusive) {
      // runs alone: wait until every other slot is idle and has freed its buffers
      if (others_run) return nullptr;
      if (request_trims(sv, i)) return nullptr;
      if (me.resident > 0) {
        me.trim_requested = true;
        return nullptr;
      }
      bool pending = false;
      for (size_t k = 0; k < sv->slots.size(); ++k)
        if (k != i && sv->slots[k]->trim_requested) pending = true;
      if (pending) return nullptr;
      *grant = sv->budget > others ? sv->budget - others : 0;
    } else {
      const uint64_t need = j.reservation;
      if (others + std::max(need, me.resident) > sv->budget) {
        if (others + need <= sv->budget) {
          me.trim_requested = true;  // fits once this slot's idle buffers are freed
          return nullptr;
        }
        request_trims(sv, i);  // idle buffers elsewhere go back to the pool
        if (j.passed_over >= kMaxPassOver) return nullptr;  // nobody passes it any more
        continue;
      }
      *grant = std::max(need, me.resident);
    }
    if (*grant == 0) return nullptr;
    std::shared_ptr<JobState> got = *it;
    for (auto p = sv->queue.begin(); p != it; ++p) (*p)->passed_over++;
    sv->queue.erase(it);
    return got;
  }
  return nullptr;
}

void finish(wg_server* sv, JobState& j, wg_status status) {
  j.status = status;
  j.phase = kDone;
  j.t_end = now_ms();
  if (status == WG_OK) sv->st.completed++;
  else if (status == WG_ERR_CANCELLED) sv->st.cancelled++;
  else sv->st.failed++;
}

// Inputs are freed stream-ordered (a plain hipFree would wait for the whole device and
// stall the other slots): on the stream of the solve that read them, or the copy stream.
void free_inputs(wg_server* sv, JobState& j, hipStream_t s) {
  if (j.d_edges) {
    (void)hipFreeAsync(j.d_edges, s ? s : sv->copy_stream);
    j.d_edges = nullptr;
    sv->core->held -= (int64_t)j.input_bytes;
  }
}

void worker(wg_server* sv, size_t i) {
  Slot& me = *sv->slots[i];
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->core->mu);
  for (;;) {
    if (me.trim_requested) {
      me.trim_requested = false;
      lk.unlock();
      wg::engine_trim(me.engine);
      lk.lock();
      me.resident = wg::engine_allocated(me.engine);
      sv->core->cv.notify_all();
      continue;
    }
    if (sv->stop && sv->queue.empty()) break;
    uint64_t grant = 0;
    std::shared_ptr<JobState> job = pick(sv, i, &grant);
    if (!job) {
      if (!me.trim_requested) sv->core->cv.wait(lk);
      continue;
    }
    JobState& j = *job;
    me.job = job;
    // (under the lock: until the solve itself starts, the engine still reports the previous
    // solve's candidates, which would hold the other slots' admissions as a long solve)
    wg::engine_clear_seen(me.engine);
    me.reservation = grant;
    me.busy_since = now_ms();
    j.phase = kRunning;
    if (j.t_start == 0) j.t_start = me.busy_since;
    uint32_t running = 0;
    for (auto& s : sv->slots) running += s->job ? 1u : 0u;
    sv->st.max_running = std::max(sv->st.max_running, running);
    wg_options o = j.opts;
    o.struct_size = sizeof(wg_options);
    o.mem_budget_bytes = me.reservation;
    lk.unlock();

    wg_result* res = nullptr;
    wg_stats stats{};
    std::vector<uint64_t> deltas(1u << 16);
    stats.delta_sizes = deltas.data();
    stats.delta_sizes_cap = deltas.size();
    wg::engine_set_cancel(me.engine, &j.cancel);
    wg_status status = j.cancel ? WG_ERR_CANCELLED
                                : wg::engine_solve(me.engine, j.query, 0, nullptr, j.d_edges,
                                                   j.d_edges + j.m, j.m, &o, me.stream, &res, &stats);
    wg::engine_set_cancel(me.engine, nullptr);
    const uint64_t peak = wg::engine_peak(me.engine);
    const std::string detail = status == WG_OK ? std::string() : std::string(wg_last_error(me.engine));
    wg_result* owned = nullptr;
    uint64_t owned_bytes = 0;
    if (status == WG_OK) {
      std::shared_ptr<Core> core = sv->core;
      status = wg::result_detach(res, me.stream, [core](uint64_t bytes) {
        std::lock_guard<std::mutex> g(core->mu);
        core->held -= (int64_t)bytes;
        core->cv.notify_all();
      }, &owned, &owned_bytes);
    }
    wg_result_free(res);

    lk.lock();
    sv->st.busy_ms += now_ms() - me.busy_since;
    me.resident = wg::engine_allocated(me.engine);
    const bool no_memory = status == WG_ERR_CAPACITY || status == WG_ERR_OUT_OF_MEMORY;
    if (no_memory && !j.cancel && !j.exclusive) {
      // outgrew its reservation while others held memory: queue it again, larger (a
      // request that failed while running alone gets no further try)
      j.requeues++;
      sv->st.requeued++;
      j.reservation = std::min<uint64_t>(sv->budget, std::max<uint64_t>(2 * me.reservation, peak + peak / 4));
      j.exclusive = j.reservation >= sv->budget / 2;  // then it waits for the whole device
      j.phase = kQueued;
      sv->queue.push_front(job);
      me.trim_requested = true;  // its buffers go back to the pool
    } else {
      if (status == WG_OK) {
        j.result = owned;
        j.stats = stats;
        j.stats.delta_sizes = nullptr;
        j.stats.delta_sizes_cap = 0;
        j.deltas.assign(deltas.begin(), deltas.begin() + std::min<uint64_t>(stats.iterations + 1, deltas.size()));
        sv->core->held += (int64_t)owned_bytes;
        // learn the memory per edge of this query kind (never below what was just seen)
        const double a = (double)peak / (double)std::max<uint64_t>(j.m, 1);
        double& al = sv->alpha[j.query == WG_QUERY_SG];
        al = std::max(0.5 * al + 0.5 * a, 0.25 * al);
      } else {
        j.error = detail;
      }
      j.peak_bytes = peak;
      free_inputs(sv, j, me.stream);
      finish(sv, j, j.cancel && status != WG_OK ? WG_ERR_CANCELLED : status);
      if (j.abandoned && j.result) {
        wg_result* r = j.result;
        j.result = nullptr;
        lk.unlock();
        wg_result_free(r);
        lk.lock();
      }
    }
    me.job.reset();
    me.reservation = 0;
    if (me.resident > sv->budget / sv->slots.size()) me.trim_requested = true;
    sv->core->cv.notify_all();
  }
  lk.unlock();
}

// Grow hook of slot i: grant `need` bytes when the budget allows, else wait for running
// solves to release memory; refuse when no other solve can make progress.
uint64_t grow(wg_server* sv, size_t i, uint64_t need) {
  std::unique_lock<std::mutex> lk(sv->core->mu);
  Slot& me = *sv->slots[i];
  const double give_up = now_ms() + kMaxMemoryWaitMs;
  for (;;) {
    const uint64_t others = usage_except(sv, i);
    if (others + need <= sv->budget) {
      const uint64_t grant = std::min(sv->budget - others, need + need / 4);
      me.reservation = grant;
      sv->core->cv.notify_all();  // idle slots held back while this solve waited
      return grant;
    }
    if (me.job && me.job->cancel) return 0;
    // can anything still free memory?  another solve that is not itself waiting, or an
    // idle slot whose buffers are (about to be) trimmed
    request_trims(sv, i);
    bool progress = false;
    for (size_t k = 0; k < sv->slots.size(); ++k) {
      const Slot& o = *sv->slots[k];
      if (k != i && ((o.job && !o.waiting_memory) || (!o.job && o.resident > 0))) progress = true;
    }
    if (!progress || now_ms() > give_up) {
      sv->core->cv.notify_all();
      return 0;
    }
    me.waiting_memory = true;
    sv->core->cv.wait_for(lk, std::chrono::milliseconds(50));
    me.waiting_memory = false;
  }
}

}  // namespace

extern "C" {

wg_status wg_server_create(int device, const wg_server_config* cfg, wg_server** out) {
  if (!out) return WG_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return WG_ERR_INVALID_ARG;
  uint32_t slots = cfg && cfg->slots ? cfg->slots : 4;
  if (slots > 16) return WG_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return WG_ERR_DEVICE;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return WG_ERR_DEVICE;
  uint64_t budget = cfg && cfg->mem_budget_bytes ? cfg->mem_budget_bytes : (uint64_t)(0.8 * (double)free_b);
  if (budget < kMinReservation) return WG_ERR_INVALID_ARG;
  wg_server* sv = new wg_server();
  sv->device = device;
  sv->budget = budget;
  sv->core = std::make_shared<Core>();
  sv->t0 = now_ms();
  sv->core->t0 = sv->t0;
  sv->st.budget_bytes = budget;
  const uint32_t hold = cfg ? cfg->hold_after_us : 0;
  sv->hold_after_ms = hold == 0xFFFFFFFFu ? -1.0 : (hold == 0 ? 8.0 : hold / 1000.0);
  if (hipStreamCreateWithFlags(&sv->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    delete sv;
    return WG_ERR_DEVICE;
  }
  sv->st.slots = slots;
  for (uint32_t i = 0; i < slots; ++i) {
    auto s = std::make_unique<Slot>();
    if (wg_engine_create(device, &s->engine) != WG_OK ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      if (s->engine) wg_engine_destroy(s->engine);
      for (auto& t : sv->slots) {
        wg_engine_destroy(t->engine);
        (void)hipStreamDestroy(t->stream);
      }
      (void)hipStreamDestroy(sv->copy_stream);
      delete sv;
      return WG_ERR_DEVICE;
    }
    s->resident = wg::engine_allocated(s->engine);
    sv->slots.push_back(std::move(s));
  }
  for (size_t i = 0; i < sv->slots.size(); ++i) {
    wg::engine_set_grow_hook(sv->slots[i]->engine, [sv, i](uint64_t need) { return grow(sv, i, need); });
    sv->slots[i]->thread = std::thread(worker, sv, i);
  }
  *out = sv;
  return WG_OK;
}

void wg_server_destroy(wg_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->core->mu);
    sv->stop = true;
    for (auto& j : sv->queue) {
      free_inputs(sv, *j, nullptr);
      finish(sv, *j, WG_ERR_CANCELLED);
    }
    sv->queue.clear();
    for (auto& s : sv->slots)
      if (s->job) s->job->cancel = true;
    sv->core->cv.notify_all();
  }
  for (auto& s : sv->slots)
    if (s->thread.joinable()) s->thread.join();
  for (auto& s : sv->slots) {
    wg_engine_destroy(s->engine);
    (void)hipStreamDestroy(s->stream);
  }
  (void)hipStreamSynchronize(sv->copy_stream);
  (void)hipStreamDestroy(sv->copy_stream);
  {
    std::lock_guard<std::mutex> g(sv->core->mu);
    sv->core->alive = false;
  }
  delete sv;
}

wg_status wg_submit(wg_server* sv, int query, const uint32_t* src, const uint32_t* dst, uint64_t m,
                    const wg_options* opts, wg_job** out) {
  if (!sv || !out || (query != WG_QUERY_TC && query != WG_QUERY_SG)) return WG_ERR_INVALID_ARG;
  *out = nullptr;
  if (m > 0 && (!src || !dst)) return WG_ERR_INVALID_ARG;
  if (opts && (opts->struct_size < 8 || opts->struct_size > sizeof(wg_options))) return WG_ERR_INVALID_ARG;
  auto j = std::make_shared<JobState>();
  j->query = query;
  j->opts.struct_size = sizeof(wg_options);
  if (opts) std::memcpy(&j->opts, opts, opts->struct_size);
  j->m = m;
  j->input_bytes = std::max<uint64_t>(8 * m, 256);
  if (hipSetDevice(sv->device) != hipSuccess) return WG_ERR_DEVICE;
  if (hipMallocAsync((void**)&j->d_edges, j->input_bytes, sv->copy_stream) != hipSuccess) {
    (void)hipGetLastError();
    return WG_ERR_OUT_OF_MEMORY;
  }
  hipError_t err = hipSuccess;
  if (m > 0) err = hipMemcpyAsync(j->d_edges, src, 4 * m, hipMemcpyDefault, sv->copy_stream);
  if (m > 0 && err == hipSuccess)
    err = hipMemcpyAsync(j->d_edges + m, dst, 4 * m, hipMemcpyDefault, sv->copy_stream);
  if (err == hipSuccess) err = hipStreamSynchronize(sv->copy_stream);
  if (err != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFreeAsync(j->d_edges, sv->copy_stream);
    return WG_ERR_INVALID_ARG;
  }
  {
    std::lock_guard<std::mutex> g(sv->core->mu);
    if (sv->stop) {
      (void)hipFreeAsync(j->d_edges, sv->copy_stream);
      return WG_ERR_INVALID_ARG;
    }
    j->t_submit = now_ms();
    j->reservation = estimate(sv, *j);
    sv->core->held += (int64_t)j->input_bytes;
    sv->queue.push_back(j);
    sv->st.submitted++;
    sv->core->cv.notify_all();
  }
  *out = new wg_job{sv, sv->core, j};
  return WG_OK;
}

wg_status wg_poll(wg_job* job, int* done) {
  if (!job || !done) return WG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(job->core->mu);
  *done = job->s->phase == kDone;
  return WG_OK;
}

wg_status wg_wait(wg_job* job, wg_result** out, wg_stats* stats) {
  if (!job) return WG_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(job->core->mu);
  JobState& j = *job->s;
  job->core->cv.wait(lk, [&] { return j.phase == kDone; });
  if (stats) {
    uint64_t* ds = stats->delta_sizes;
    const uint64_t dc = stats->delta_sizes_cap;
    *stats = j.stats;
    stats->delta_sizes = ds;
    stats->delta_sizes_cap = dc;
    if (ds)
      for (uint64_t k = 0; k < dc && k < j.deltas.size(); ++k) ds[k] = j.deltas[k];
  }
  if (out) {
    *out = nullptr;
    if (j.status == WG_OK) {
      if (j.result_taken) return WG_ERR_INVALID_ARG;
      *out = j.result;
      j.result_taken = true;
    }
  }
  return j.status;
}

wg_status wg_cancel(wg_job* job) {
  if (!job) return WG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(job->core->mu);
  JobState& j = *job->s;
  if (!job->core->alive) return WG_OK;  // the server is gone: the job is done
  wg_server* sv = job->server;
  j.cancel = true;
  if (j.phase == kQueued) {
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
      if (it->get() == &j) {
        sv->queue.erase(it);
        break;
      }
    free_inputs(sv, j, nullptr);
    finish(sv, j, WG_ERR_CANCELLED);
    sv->core->cv.notify_all();
  }
  return WG_OK;
}

wg_status wg_job_get_info(const wg_job* job, wg_job_info* info) {
  if (!job || !info) return WG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(job->core->mu);
  const JobState& j = *job->s;
  const double t0 = job->core->t0;
  std::memset(info, 0, sizeof(*info));
  info->status = j.status;
  info->phase = (uint32_t)j.phase;
  info->query = (uint32_t)j.query;
  info->requeues = j.requeues;
  info->reservation_bytes = j.reservation;
  info->peak_bytes = j.peak_bytes;
  info->submit_ms = j.t_submit - t0;
  info->start_ms = j.t_start > 0 ? j.t_start - t0 : 0;
  info->end_ms = j.t_end > 0 ? j.t_end - t0 : 0;
  return WG_OK;
}

void wg_job_free(wg_job* job) {
  if (!job) return;
  wg_result* leftover = nullptr;
  {
    std::lock_guard<std::mutex> g(job->core->mu);
    JobState& j = *job->s;
    wg_server* sv = job->core->alive ? job->server : nullptr;
    if (j.phase != kDone && sv) {
      j.cancel = true;
      j.abandoned = true;
      if (j.phase == kQueued) {
        for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
          if (it->get() == &j) {
            sv->queue.erase(it);
            break;
          }
        free_inputs(sv, j, nullptr);
        finish(sv, j, WG_ERR_CANCELLED);
      }
    } else if (j.phase == kDone && j.result && !j.result_taken) {
      leftover = j.result;
      j.result_taken = true;
    }
    job->core->cv.notify_all();
  }
  wg_result_free(leftover);  // a running job's result is freed by the worker's job record
  delete job;
}

wg_status wg_server_get_stats(const wg_server* sv, wg_server_stats* out) {
  if (!sv || !out) return WG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(sv->core->mu);
  *out = sv->st;
  out->held_bytes = (uint64_t)std::max<int64_t>(sv->core->held, 0);
  out->queued = (uint32_t)sv->queue.size();
  return WG_OK;
}

}  // extern "C"
