// Engine entry points used by the request server (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <functional>

#include "../../include/wg.h"

namespace wg {

// Asked by an engine whose next allocation would exceed its budget, with the total it
// needs.  Returns the new budget (>= need) or 0 to refuse (the solve then fails with
// WG_ERR_CAPACITY).  May block until memory frees up.
using GrowHook = std::function<uint64_t(uint64_t need)>;

// wg_tc / wg_sg (num == 0) or their batched forms.
wg_status engine_solve(wg_engine* e, int query, uint32_t num, const uint64_t* d_offsets,
                       const uint32_t* src, const uint32_t* dst, uint64_t m, const wg_options* o,
                       void* stream, wg_result** out, wg_stats* st);
uint64_t engine_allocated(const wg_engine* e);
uint64_t engine_peak(const wg_engine* e);  // high-water mark of the latest solve
void engine_trim(wg_engine* e);            // free the relation buffers; results of the engine go stale
void engine_set_grow_hook(wg_engine* e, GrowHook hook);
// While set, the solve stops at its next host check with WG_ERR_CANCELLED once *flag holds.
void engine_set_cancel(wg_engine* e, const std::atomic<bool>* flag);
// The largest per-iteration candidate count the solve in progress has read back at its
// host checks (0 before the first; reset when a solve starts).  Any thread may read it.
uint64_t engine_seen_candidates(const wg_engine* e);
// Forget the previous solve's sizes now, before the next solve starts (a caller that hands
// the engine a new job reads engine_seen_candidates of that job from then on).
void engine_clear_seen(wg_engine* e);

// Copy a result's keys (stream-ordered, then waits) into a device buffer owned by a new
// handle.  `release(bytes)` runs when that handle is freed.
wg_status result_detach(const wg_result* r, hipStream_t s, std::function<void(uint64_t)> release,
                        wg_result** out, uint64_t* bytes);

// Detail of the latest failure of a call that takes no engine (wg_last_error(NULL) returns
// it; one per host thread).
void set_call_error(const char* msg);

}  // namespace wg
