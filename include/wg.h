/*
 * wg.h -- C ABI of the MI355X semi-naive fixpoint engine (TC and SG).
 *
 * The engine evaluates two Datalog programs over a directed edge relation E of
 * (uint32 src, uint32 dst) pairs and returns the least fixpoint as a
 * lexicographically sorted, duplicate-free pair array:
 *
 *   TC  T(x,y) <- E(x,y).            T(x,z) <- T(x,y), E(y,z).
 *       (paper Section II, the running example)
 *   SG  SG(x,y) <- E(p,x), E(p,y), x != y.
 *       SG(x,y) <- E(a,x), SG(a,b), E(b,y).
 *       (paper Section VI, same-generation; E is oriented parent -> child)
 *
 * Evaluation is semi-naive (Section II, "Semi-Naive Evaluation"): Delta^0 = Full =
 * the base facts; iteration i joins Delta^{i-1} with E, sorts the candidates,
 * drops duplicates and tuples already in Full, merges the survivors Delta^i into
 * Full and stops at the first empty Delta^i.  Every stage runs in HIP kernels on
 * one GPU and the loop stays on the device between batch boundaries
 * (Section V-B: the host only learns when the fixpoint terminates).
 *
 * Conventions shared by every entry point:
 *  - Every call returns wg_status; nothing throws, aborts or exits across the ABI.
 *  - Pointers named d_* are device pointers on the engine's device.  Host pointers
 *    are accepted only where a comment says so.
 *  - `stream` is a hipStream_t of the engine's device (NULL = the null stream).
 *    Calls are ordered on it.  Input arrays are read before the call returns.
 *  - Input edges are a multiset in any order.  Duplicates collapse; self-loops are
 *    ordinary edges; any uint32 id is valid (no sentinel values).  m = 0 gives an
 *    empty result.
 *  - Results are exact: one byte string per input, independent of batch sizes,
 *    loop mode or launch shapes.
 *  - On error no result is produced and *out stays NULL.  The engine stays usable
 *    after every status except WG_ERR_DEVICE.
 *  - An engine is not thread-safe; use one engine per host thread / stream.
 */
#ifndef WG_H_
#define WG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WG_OK = 0,
  WG_ERR_INVALID_ARG = 1,   /* bad pointer, size or option */
  WG_ERR_OUT_OF_MEMORY = 2, /* the device allocator failed */
  WG_ERR_CAPACITY = 3,      /* the fixpoint needs more device memory than mem_budget_bytes */
  WG_ERR_DEVICE = 4,        /* a HIP call failed or a device wait expired; destroy the engine */
  WG_ERR_ITER_LIMIT = 5,    /* max_iterations reached before the fixpoint */
  WG_ERR_STALE = 6,         /* the result belongs to an earlier solve of this engine */
  WG_ERR_CANCELLED = 7      /* a served request was cancelled */
} wg_status;

typedef enum { WG_QUERY_TC = 0, WG_QUERY_SG = 1, WG_QUERY_TRIANGLES = 2 } wg_query;

/* wg_options.flags */
#define WG_SG_IRREFLEXIVE 0x1u /* SG: drop (x,x) from the final relation */
#define WG_STAGE_TIMING 0x2u   /* time every kernel launch with HIP events (fills stage_ms) */
#define WG_NO_SPECULATION 0x4u /* enqueue nothing behind a batch while the host checks it */
#define WG_JOIN_HASH 0x8u      /* TC and triangles: join through a linear-probing hash table of
                                  E (thread per tuple) instead of the binary-search join of
                                  Section IV-A -- the baseline of the paper's comparison */
#define WG_UNFUSED_DEDUP 0x10u /* ablation of Section IV-B's fusion: deduplicate the sorted
                                  candidates in one compaction pass, then take the set
                                  difference with Full in a second (same result) */
#define WG_JOIN_HASH_ROWS 0x100u /* TC and triangles: the sorted join with its row lookups
                                   through a hash table of E's distinct rows (row -> index of
                                   its contiguous edges) instead of the index; triangles probe
                                   each closing edge in a hash set of E's pairs -- the fair hash
                                   baseline: O(1) expected per lookup, the emit load-balanced as
                                   the sorted join's (one thread per output, not per tuple) */
#define WG_SPARSE_INDEX 0x20u /* index the edge rows by bisection over the distinct rows even
                                 where the row ids span a range small enough for the dense
                                 index (one array entry per row id) the engine would use */
#define WG_ITER_GRAPH 0x40u   /* record one iteration's launches once as a HIP graph and replay
                                 it, instead of launching every kernel from the host (the
                                 default; on MI355X both take the same time, since a loop
                                 kernel's own latency, not its launch, bounds small iterations) */
#define WG_LSD_SORT 0x80u     /* TC: sort every iteration's candidates with the LSD passes of
                                 Section V-C and take the difference with the compaction of
                                 Section IV-B, never with the segmented sort or the row pass
                                 (which sort only each source row's run, the join having
                                 emitted the candidates grouped by row) */
#define WG_NO_TAIL_LOOP 0x200u /* WG_LOOP_AUTO without its tail loop: every iteration from the
                                  host-enqueued multi-block launches (ablation) */

/* wg_options.loop_mode */
#define WG_LOOP_AUTO 0u     /* the default: device-resident loop checked by the host every 2
                               iterations (batch_k overrides), with a speculative batch
                               enqueued behind every check; and once the delta (at most
                               1,024-4,096 tuples by key width and query) and an
                               iteration's candidates (at most 4,096) fit one block, one
                               launch runs the fixpoint's tail: a single workgroup loops
                               over whole iterations (join, sort, dedup + difference,
                               merge) until the fixpoint, the iteration limit or an
                               iteration that outgrows it, which goes back to the
                               multi-block launches (Section V-B's device-resident loop
                               carried into one launch).  TC and SG; not with
                               WG_JOIN_HASH, WG_JOIN_HASH_ROWS, WG_UNFUSED_DEDUP or
                               WG_NO_TAIL_LOOP */
#define WG_LOOP_BATCHED 1u  /* K iterations per host check (Section V-B, batched recording);
                               batch_k = 0 takes the paper's policy: K = 30 halving for
                               TC, 10 for SG */
#define WG_LOOP_HOST 2u     /* one host check per iteration (K = 1); reference mode */
#define WG_LOOP_STAGE 3u    /* ablation of Section V-B: K = 1 plus a blocking host read of
                               the candidate count after the join count and of the delta
                               size after the compaction, as a loop that sizes each stage
                               from the host would do (three host round trips per
                               iteration; the kernels still size themselves on the device) */

typedef struct {
  uint32_t struct_size;      /* sizeof(wg_options); older sizes are accepted */
  uint32_t flags;            /* WG_SG_IRREFLEXIVE, WG_STAGE_TIMING, ... (above) */
  uint32_t batch_k;          /* iterations per host check; 0 = the loop mode's default
                                (WG_LOOP_BATCHED: 30 with halving for TC, 10 for SG, as in
                                Section V-B's adaptive batch sizing) */
  uint32_t loop_mode;        /* WG_LOOP_* */
  uint32_t radix_field_bits; /* 0 = the bit length of the largest id (Section V-C adapts
                                the width; it rounds to 16, 24 or 32); else 1..32 bits,
                                which must cover the largest id */
  uint32_t timing_stages;    /* with WG_STAGE_TIMING: bitmask of WG_STAGE_* kinds to time
                                (0 = all); events cost launch overlap, so time few kinds */
  uint64_t max_iterations;   /* 0 = unlimited */
  uint64_t mem_budget_bytes; /* 0 = no limit beyond the device allocator */
  uint64_t force_overflow_at_iter; /* test hook: report a capacity overflow once at this
                                      iteration (1-based) to exercise grow-and-resume */
  uint32_t radix_digit_bits; /* 0 = the engine's choice (default 8, or autotuned); else
                                8..11 bits per LSD pass: ceil(2w / bits) passes */
  uint32_t tile_items;       /* 0 = the engine's choice; 8 = small sort tile; 12 or 16 =
                                large tile (16 keys per thread for 32-bit keys, 12 for
                                64-bit keys) */
} wg_options;

/* Kernel kinds reported in wg_stats.stage_ms / stage_launches / stage_bytes. */
enum {
  WG_STAGE_JOIN_COUNT = 0, /* binary-search range lookup + count scan (Section IV-A) */
  WG_STAGE_JOIN_EMIT = 1,  /* candidate emission into scanned slabs (Section IV-A); also
                              the one-block join + sort of a small iteration */
  WG_STAGE_RADIX_HIST = 2, /* per-block digit counts and their scan, one per LSD pass
                              (Section V-C); also the one-block sort of a small input */
  WG_STAGE_RADIX_PASS = 3, /* the stable scatter of one LSD pass (Section V-C) */
  WG_STAGE_DEDUP_DIFF = 4, /* fused dedup + set difference (Section IV-B) */
  WG_STAGE_MERGE = 5,      /* disjoint merge-path merge (Section IV-C) */
  WG_STAGE_PREPARE = 6,    /* max-id scan, packing, edge index, result unpack */
  WG_STAGE_SEG_SORT = 7,   /* TC: the segmented sort of a join's row-grouped candidates */
  WG_STAGE_ROW_DIFF = 8,   /* TC: the row pass -- sort, dedup and difference of each row of the
                              join's row-grouped candidates in one LDS bitmap (Sections IV-B,
                              V-C), which replaces the sort and the compaction of a large
                              iteration */
  WG_STAGE_TAIL_LOOP = 9,  /* the one-block launch that runs the fixpoint's tail
                              (its fold into run B is timed as WG_STAGE_MERGE) */
  WG_NUM_STAGES = 10
};

typedef struct {
  uint64_t iterations;      /* join rounds, including the one that found the empty delta */
  uint64_t result_tuples;   /* |fixpoint| */
  uint64_t base_tuples;     /* |Delta^0| */
  uint64_t join_candidates; /* candidates summed over iterations, with multiplicity */
  uint64_t host_syncs;      /* host waits on the device during the call */
  uint64_t resumes;         /* grow-and-resume cycles after a capacity overflow */
  uint32_t field_bits;      /* radix field width used (bits per id) */
  uint32_t key_bytes;       /* bytes per packed key (4 or 8) */
  double solve_ms;          /* host wall clock of the call */
  double stage_ms[WG_NUM_STAGES];        /* with WG_STAGE_TIMING: summed kernel time */
  uint64_t stage_launches[WG_NUM_STAGES];
  uint64_t stage_bytes[WG_NUM_STAGES];   /* algorithmic HBM bytes of each kernel kind */
  uint64_t* delta_sizes;    /* optional caller HOST buffer: |Delta^0| .. |Delta^iterations| */
  uint64_t delta_sizes_cap; /* its capacity in entries (filled up to the capacity) */
  uint32_t digit_bits;      /* radix digit bits per LSD pass used */
  uint32_t sort_passes;     /* LSD passes per sort: ceil(key bits / digit_bits) */
  uint64_t tail_iterations; /* iterations run inside tail-loop launches */
} wg_stats;

typedef struct wg_engine wg_engine; /* per device: buffers, control block, sort tuning table */
typedef struct wg_result wg_result; /* a device-resident fixpoint owned by the caller */

/* Device memory for an engine's buffers (the boundary's allocator hook; Section V-C keeps
 * every relation and its ping-pong partner resident in device memory, and this hook lets a
 * caller -- e.g. a framework's caching allocator -- supply that memory).
 *
 *  alloc(bytes, stream, user): return `bytes` of device memory of the engine's device,
 *      usable by work enqueued on `stream` (a hipStream_t; NULL is the null stream) from
 *      this point on, or NULL when none is available (the call in progress then fails with
 *      WG_ERR_OUT_OF_MEMORY and leaves the engine usable).
 *  free(ptr, bytes, stream, user): the engine's last use of `ptr` is enqueued on `stream`
 *      before this call (or has finished); the memory must not be handed to work that is
 *      not ordered after that point on `stream`.  `bytes` is what alloc was asked for.
 *
 * Both are called on the thread that called into the engine, during wg_engine_create_ex,
 * the solve calls (buffers grow on demand) and wg_engine_destroy; never concurrently for
 * one engine.  Neither may call into the engine. */
typedef struct {
  void* (*alloc)(uint64_t bytes, void* stream, void* user);
  void (*free)(void* ptr, uint64_t bytes, void* stream, void* user);
  void* user;
} wg_allocator;

/* Create an engine on HIP device `device`.  Allocates the control block and the sort's
 * count arrays; relation buffers grow on demand and are reused across calls.  An engine
 * serves one host thread at a time.  `allocator` (nullable; copied) supplies every device
 * allocation of the engine; NULL takes the device's stream-ordered pool (hipMallocAsync /
 * hipFreeAsync on the stream of the call), so growing or releasing a buffer never waits for
 * other streams.  WG_ERR_INVALID_ARG: a non-null allocator without both functions, or no
 * such device; WG_ERR_OUT_OF_MEMORY: the allocator failed. */
wg_status wg_engine_create_ex(int device, const wg_allocator* allocator, wg_engine** out);

/* wg_engine_create_ex(device, NULL, out). */
wg_status wg_engine_create(int device, wg_engine** out);

/* Free every device allocation of the engine (through its allocator, after waiting for the
 * device).  Results of the engine become invalid. */
void wg_engine_destroy(wg_engine* engine);

/* Transitive closure of the m edges (d_src[i], d_dst[i]) (Section II; semi-naive loop,
 * Sections IV and V).  On WG_OK *out holds the fixpoint; stats (nullable) is filled. */
wg_status wg_tc(wg_engine* engine, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* options, void* stream, wg_result** out, wg_stats* stats);

/* Same-generation fixpoint of the m edges, E(parent, child) (Section VI). */
wg_status wg_sg(wg_engine* engine, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                const wg_options* options, void* stream, wg_result** out, wg_stats* stats);

/* Batched fixpoints: `num_instances` independent instances laid out back to back.
 * Instance i owns edges d_offsets[i] .. d_offsets[i+1] of (d_src, d_dst); its vertex ids
 * are local to it.  d_offsets (device, num_instances + 1 entries) starts at 0, does not
 * decrease and ends at m, else WG_ERR_INVALID_ARG.  The instances run as one fixpoint
 * over their disjoint union: every key carries the instance in its top bits
 * (instance | src | dst), so one launch sequence serves all of them and the loop ends
 * when every instance has reached its fixpoint (iterations = the largest instance's).
 * The instance bits plus the id field must fit 32 bits (e.g. 4096 instances of up to
 * 65,536 vertices).  The result holds every instance's fixpoint, sorted by (instance,
 * src, dst), with local ids; wg_result_offsets gives the instance boundaries.  This
 * packing of many graphs into one solve is an addition to the paper's method, which
 * evaluates one query at a time. */
wg_status wg_tc_batch(wg_engine* engine, uint32_t num_instances, const uint64_t* d_offsets,
                      const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                      const wg_options* options, void* stream, wg_result** out, wg_stats* stats);
wg_status wg_sg_batch(wg_engine* engine, uint32_t num_instances, const uint64_t* d_offsets,
                      const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                      const wg_options* options, void* stream, wg_result** out, wg_stats* stats);

/* Instances of the result (1 for wg_tc / wg_sg). */
uint32_t wg_result_instances(const wg_result* result);

/* Instance boundaries of the result: offsets_out[i] = first tuple of instance i,
 * offsets_out[instances] = wg_result_size.  offsets_out is a device or a host pointer
 * (then the call waits) with capacity >= instances + 1 entries. */
wg_status wg_result_offsets(const wg_result* result, uint64_t* offsets_out, uint64_t capacity,
                            void* stream);

/* Triangle counting (Section VI): the number of bindings (a, b, c) of
 * triangle(a,b,c) <- edge(a,b), edge(b,c), edge(c,a) over the set of the m edges
 * (d_src[i], d_dst[i]) -- a directed 3-cycle counts once per rotation, an edge (a, a)
 * counts once as (a, a, a) -- which equals trace(A^3) of the 0/1 adjacency matrix.  One
 * non-recursive pass of the sorted-array join: every edge (a, b) expands the row of b in
 * E, and each two-path (a, c) is probed against E for (c, a); nothing is materialised.
 * *count_out (host) receives the count.  More than 2^32 two-paths: WG_ERR_CAPACITY.
 * stats.join_candidates is the number of two-paths. */
wg_status wg_triangles(wg_engine* engine, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                       const wg_options* options, void* stream, uint64_t* count_out,
                       wg_stats* stats);

/* Kernel-level entry points: single stages of the hot path on caller arrays, for
 * measuring them apart from a fixpoint (sizes and key widths of the caller's choosing).
 *
 * wg_sort_keys (Section V-C): sorts the n keys of d_keys (device; key_bytes 4 or 8 per
 * key, every key below 2^key_bits) ascending, in place, with the LSD passes -- count,
 * scan and scatter launches per pass of the engine's sort configuration for that key
 * width (wg_get_sort_config), ceil(key_bits / digit bits) passes.  d_tmp (device, n keys,
 * caller-owned) is the ping-pong buffer; with an odd pass count the result is copied back
 * into d_keys.  Neither the one-block sort nor the segmented sort is used.
 *
 * wg_merge_keys (Section IV-C): d_out[0, na + nb) = the merge of the ascending runs
 * d_a[0, na) and d_b[0, nb) (device, key_bytes per key; d_out caller-owned and disjoint
 * from both; on equal keys A's come first).
 *
 * Both run on `stream` (NULL: the default stream) and return after enqueueing.  options
 * (nullable): only WG_STAGE_TIMING is read; with it, stats (nullable) receives the summed
 * kernel times, launches and algorithmic bytes per kernel kind (radix count, radix
 * scatter; merge), after a synchronisation.  The engine's current result stays valid.
 * WG_ERR_INVALID_ARG: a null array with n > 0, key_bytes not 4 or 8, key_bits outside
 * 1..8*key_bytes, more than 2^32 - 16 keys. */
wg_status wg_sort_keys(wg_engine* engine, void* d_keys, void* d_tmp, uint64_t n, uint32_t key_bytes,
                       uint32_t key_bits, const wg_options* options, void* stream, wg_stats* stats);
wg_status wg_merge_keys(wg_engine* engine, const void* d_a, uint64_t na, const void* d_b, uint64_t nb,
                        void* d_out, uint32_t key_bytes, const wg_options* options, void* stream,
                        wg_stats* stats);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: wg_sort_keys without an engine and
 * without any allocation.  Sorts the n keys of d_keys (device; key_bytes 4 or 8 per key,
 * every key below 2^key_bits) ascending in place with the same LSD passes (8-bit digits,
 * the engine's default tiles, up to 1,024 blocks); d_tmp (device, n keys, caller-owned) is
 * the ping-pong buffer, as for wg_sort_keys.  Its scratch (control block, per-block digit
 * counts, digit totals; WG_SORT_NOALLOC_SCRATCH_BYTES) is a static array of the library,
 * one per device, held until the process ends: the call itself allocates nothing and only
 * enqueues kernels (and, for an odd pass count, one device-to-device copy) on `stream`
 * (NULL: the null stream) of the current device, returning before they run.  Calls on one
 * device share that scratch: calls whose work overlaps on the device (different streams
 * not ordered against each other) race and give wrong results; calls in stream order are
 * safe (each rewrites the whole control block first).
 * WG_ERR_INVALID_ARG: key_bytes not 4 or 8, key_bits outside 1..8*key_bytes, more than
 * 2^32 - 16 keys, or a NULL array with n > 0; WG_ERR_DEVICE: no usable current device or a
 * failed launch.  wg_last_error(NULL) gives the detail (per host thread). */
#define WG_SORT_NOALLOC_SCRATCH_BYTES 1049856u
wg_status wg_sort_keys_noalloc(void* d_keys, void* d_tmp, uint64_t n, uint32_t key_bytes, uint32_t key_bits,
                               void* stream);

/* Synchronisation costs behind the loop policies of Section V-B, for the ablation that
 * weighs a persistent launch against launches per stage.  barrier_us: one grid-wide barrier
 * inside a single cooperative launch of `blocks` workgroups of 256 threads, every block
 * arriving on one counter (a launch with `rounds` barriers against one with none);
 * barrier2_us: the same with two levels, blocks arriving on one of 8 group counters (the
 * device's XCDs, to which consecutive blocks are dealt in turn) and each group's last block
 * on the top counter; barrier_cg_us: the runtime's own grid synchronisation for
 * cooperative launches (cooperative groups' grid sync); launch_us: one kernel boundary (min(rounds, 512) empty launches of
 * the same shape back to back on one in-order stream, all queued behind a 20 ms delay
 * kernel before the timed window opens, so that the host's launch rate does not enter it).
 * Microseconds per event, timed with HIP events on a stream of the call's own on `device`.
 * The call allocates a few KB of device memory, waits for its work (about 20 ms longer than
 * the events it times), frees everything and leaves the calling thread's current device as
 * it found it.
 * WG_ERR_INVALID_ARG: a NULL output, blocks outside 1..2048 or beyond what can be resident
 * at once on the device, rounds outside 1..1,000,000, or no such device;
 * WG_ERR_DEVICE: no cooperative launch on the device, a failed launch, or a wait of the
 * probe's own barriers that gave up (those waits are bounded, so their launches always end).
 */
wg_status wg_probe_sync_costs(int device, uint32_t blocks, uint32_t rounds, double* barrier_us,
                              double* barrier2_us, double* barrier_cg_us, double* launch_us);

/* Number of tuples in the result (for a batch: over all instances). */
uint64_t wg_result_size(const wg_result* result);

/* Unpack the result into split arrays src_out[0..n), dst_out[0..n), n = wg_result_size,
 * lexicographically sorted.  Both pointers are device pointers, or both host pointers
 * (then the call waits for the copy).  capacity is the length of each array.
 * Returns WG_ERR_STALE when the engine has started another solve since. */
wg_status wg_result_copy(const wg_result* result, uint32_t* src_out, uint32_t* dst_out,
                         uint64_t capacity, void* stream);

/* Release a result handle.  An engine's result lives in the engine's buffers until its
 * next solve; a served result owns a device copy, freed in order on the null stream
 * (after copies enqueued on blocking streams). */
void wg_result_free(wg_result* result);

/* ----- Sort configuration and the autotuner (radix digit width and tile size).
 * The engine keeps one configuration per key type (32-bit keys when 2w + instance bits
 * <= 32, else 64-bit).  Defaults: 8-bit digits (Section V-C), large tile, 4 blocks per
 * compute unit.  Results never depend on the configuration, only time does. */
typedef struct {
  uint32_t digit_bits; /* 8..11 bits per LSD pass */
  uint32_t tile_items; /* keys per thread: 8 (small tile), 16 (32-bit keys) or 12 (64-bit) */
  uint32_t blocks;     /* blocks of each count and scatter launch, 1..2048 */
  uint32_t reserved;
} wg_sort_config;

#define WG_TUNE_MAX_TRIALS 64
typedef struct {
  uint32_t trials;        /* configurations timed (besides the one in use before) */
  uint32_t key_bytes;     /* key type the installed configuration applies to */
  wg_sort_config best;    /* the configuration installed */
  double best_ms;         /* its solve time: minimum over the timed repetitions */
  double before_ms;       /* the same for the configuration in use before the call */
  wg_sort_config tried[WG_TUNE_MAX_TRIALS];
  double tried_ms[WG_TUNE_MAX_TRIALS];
} wg_tune_report;

wg_status wg_get_sort_config(const wg_engine* engine, uint32_t key_bytes, wg_sort_config* out);
wg_status wg_set_sort_config(wg_engine* engine, uint32_t key_bytes, const wg_sort_config* config);

/* Autotuner: solve the given query (num_instances = 0 with d_offsets = NULL: a single
 * instance, else a batch as in wg_tc_batch) once per candidate configuration -- digit
 * bits 8..11 x small or large tile x 2, 4 or 8 blocks per compute unit -- `repeats` timed
 * times each after one warm-up (0 = 2), and install the fastest for the solve's key
 * type, keeping the current one unless another is faster.  options' digit and tile
 * fields are ignored.  report (nullable, host) receives every timing. */
wg_status wg_autotune(wg_engine* engine, int query, uint32_t num_instances, const uint64_t* d_offsets,
                      const uint32_t* d_src, const uint32_t* d_dst, uint64_t m,
                      const wg_options* options, uint32_t repeats, void* stream,
                      wg_tune_report* report);

/* ----- Serving: a request server with continuous batching (an addition to the paper's
 * method, which evaluates one query at a time).
 *
 * The server owns `slots` engines, each with a worker thread and its own HIP stream, so
 * the solves of different slots overlap on the device.  Requests queue up and are
 * admitted to a free slot as soon as the device-memory budget allows: each reserves an
 * estimate of its peak memory (bytes per edge, learned per query kind from finished
 * solves).  The reservations of running solves, the buffers idle engines keep, resident
 * results and queued inputs stay within mem_budget_bytes.  A solve that outgrows its
 * reservation asks for more and waits while others hold the memory; when every running
 * solve is waiting, the youngest gives up and is queued again with a larger reservation
 * (the whole budget if need be: it then runs alone).  A request larger than the whole
 * budget fails with WG_ERR_CAPACITY.  Results stay on the device until freed.  Each
 * result is the same bytes as wg_tc / wg_sg on the same input alone.  Functions of one
 * server may be called from any host threads. */
typedef struct wg_server wg_server;
typedef struct wg_job wg_job;

typedef struct {
  uint32_t slots;            /* concurrent solves, 1..16; 0 = 4 */
  /* Long-solve hold: while a solve has run longer than this (microseconds), or has shown
   * an iteration of 2^21 candidates or more at one of its host checks, no further request
   * is admitted until it ends, so that the heavy tail of a mix runs nearly alone instead
   * of slowing down beside new arrivals (tail latency); 0 = the default, 8000;
   * 0xFFFFFFFF = never hold. */
  uint32_t hold_after_us;
  uint64_t mem_budget_bytes; /* device memory of all slots, results and inputs; 0 = 80% of free */
} wg_server_config;

typedef struct {
  uint64_t submitted, completed, failed, cancelled, requeued;
  uint32_t slots;
  uint32_t max_running;   /* most solves that ran at once */
  uint32_t queued;        /* requests waiting now */
  uint32_t reserved;
  uint64_t budget_bytes;
  uint64_t held_bytes;    /* resident results and queued inputs now */
  double busy_ms;         /* summed wall time of all solves */
} wg_server_stats;

typedef struct {
  wg_status status;       /* final status once phase == 2 */
  uint32_t phase;         /* 0 queued, 1 running, 2 done */
  uint32_t query;         /* WG_QUERY_* */
  uint32_t requeues;      /* times the request was queued again with a larger reservation */
  uint64_t reservation_bytes;
  uint64_t peak_bytes;    /* engine memory high-water mark of the solve */
  double submit_ms, start_ms, end_ms; /* server clock (ms since wg_server_create) */
} wg_job_info;

wg_status wg_server_create(int device, const wg_server_config* config /* nullable */,
                           wg_server** out);
/* Cancels queued requests, lets running solves stop at their next host check, joins the
 * workers.  Results already handed out stay valid until freed. */
void wg_server_destroy(wg_server* server);

/* Queue a TC or SG solve of m edges.  src / dst are device or host pointers; they are
 * copied (on a stream of the server) before the call returns, so device inputs must be
 * complete when it is made.  options as for wg_tc (mem_budget_bytes is set by the
 * server). */
wg_status wg_submit(wg_server* server, int query, const uint32_t* src, const uint32_t* dst,
                    uint64_t m, const wg_options* options, wg_job** out);
wg_status wg_poll(wg_job* job, int* done);
/* Block until the request is done; returns its status.  On WG_OK *out (nullable) receives
 * the result, which the caller frees with wg_result_free (once per job). */
wg_status wg_wait(wg_job* job, wg_result** out, wg_stats* stats);
/* A queued request ends at once with WG_ERR_CANCELLED; a running one at its next host
 * check. */
wg_status wg_cancel(wg_job* job);
wg_status wg_job_get_info(const wg_job* job, wg_job_info* info);
/* Release the handle (cancels the request if it has not finished). */
void wg_job_free(wg_job* job);
wg_status wg_server_get_stats(const wg_server* server, wg_server_stats* out);

/* Static text for a status code. */
const char* wg_status_string(wg_status status);

/* Detail of the most recent failure on the engine ("" if none); NULL: of the latest call
 * that takes no engine on this host thread (wg_sort_keys_noalloc). */
const char* wg_last_error(const wg_engine* engine);

#ifdef __cplusplus
}
#endif

#endif /* WG_H_ */
