"""ctypes binding of the C ABI in include/wg.h.

The functions named like the C entry points (``wg_tc``, ``wg_sg``, ``wg_result_copy``
...) only marshal arguments; every step of the fixpoint runs in the HIP library.
``tc`` / ``sg`` are conveniences over them that take and return torch tensors on the
GPU (torch supplies device memory and the stream, nothing else).

The library must be built (``python -m paper_2607_17571_amd.build``); importing this
module does not build it, and every call fails loudly when it is missing.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwg.so")

WG_OK = 0
WG_ERR_INVALID_ARG = 1
WG_ERR_OUT_OF_MEMORY = 2
WG_ERR_CAPACITY = 3
WG_ERR_DEVICE = 4
WG_ERR_ITER_LIMIT = 5
WG_ERR_STALE = 6
WG_ERR_CANCELLED = 7

WG_SG_IRREFLEXIVE = 0x1
WG_STAGE_TIMING = 0x2
WG_NO_SPECULATION = 0x4
WG_JOIN_HASH = 0x8
WG_JOIN_HASH_ROWS = 0x100
WG_NO_TAIL_LOOP = 0x200
WG_UNFUSED_DEDUP = 0x10
WG_SPARSE_INDEX = 0x20
WG_ITER_GRAPH = 0x40
WG_LSD_SORT = 0x80

WG_QUERY_TC = 0
WG_QUERY_SG = 1
WG_QUERY_TRIANGLES = 2

WG_LOOP_AUTO = 0
WG_LOOP_BATCHED = 1
WG_LOOP_HOST = 2
WG_LOOP_STAGE = 3

STAGES = ["join_count", "join_emit", "radix_hist", "radix_pass", "dedup_diff", "merge", "prepare",
          "seg_sort", "row_diff", "tail_loop"]
WG_NUM_STAGES = len(STAGES)


class WgOptions(ctypes.Structure):
    _fields_ = [
        ("struct_size", c_uint32),
        ("flags", c_uint32),
        ("batch_k", c_uint32),
        ("loop_mode", c_uint32),
        ("radix_field_bits", c_uint32),
        ("timing_stages", c_uint32),
        ("max_iterations", c_uint64),
        ("mem_budget_bytes", c_uint64),
        ("force_overflow_at_iter", c_uint64),
        ("radix_digit_bits", c_uint32),
        ("tile_items", c_uint32),
    ]


class WgStats(ctypes.Structure):
    _fields_ = [
        ("iterations", c_uint64),
        ("result_tuples", c_uint64),
        ("base_tuples", c_uint64),
        ("join_candidates", c_uint64),
        ("host_syncs", c_uint64),
        ("resumes", c_uint64),
        ("field_bits", c_uint32),
        ("key_bytes", c_uint32),
        ("solve_ms", c_double),
        ("stage_ms", c_double * WG_NUM_STAGES),
        ("stage_launches", c_uint64 * WG_NUM_STAGES),
        ("stage_bytes", c_uint64 * WG_NUM_STAGES),
        ("delta_sizes", POINTER(c_uint64)),
        ("delta_sizes_cap", c_uint64),
        ("digit_bits", c_uint32),
        ("sort_passes", c_uint32),
        ("tail_iterations", c_uint64),
    ]


class WgSortConfig(ctypes.Structure):
    _fields_ = [("digit_bits", c_uint32), ("tile_items", c_uint32), ("blocks", c_uint32),
                ("reserved", c_uint32)]

    def as_dict(self) -> dict:
        return {"digit_bits": int(self.digit_bits), "tile_items": int(self.tile_items),
                "blocks": int(self.blocks)}


WG_TUNE_MAX_TRIALS = 64


class WgTuneReport(ctypes.Structure):
    _fields_ = [
        ("trials", c_uint32),
        ("key_bytes", c_uint32),
        ("best", WgSortConfig),
        ("best_ms", c_double),
        ("before_ms", c_double),
        ("tried", WgSortConfig * WG_TUNE_MAX_TRIALS),
        ("tried_ms", c_double * WG_TUNE_MAX_TRIALS),
    ]

    def as_dict(self) -> dict:
        return {"key_bytes": int(self.key_bytes), "best": self.best.as_dict(),
                "best_ms": float(self.best_ms), "before_ms": float(self.before_ms),
                "trials": [dict(self.tried[i].as_dict(), ms=float(self.tried_ms[i]))
                           for i in range(int(self.trials))]}


class WgServerConfig(ctypes.Structure):
    _fields_ = [("slots", c_uint32), ("hold_after_us", c_uint32), ("mem_budget_bytes", c_uint64)]


class WgServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("completed", c_uint64), ("failed", c_uint64),
                ("cancelled", c_uint64), ("requeued", c_uint64), ("slots", c_uint32),
                ("max_running", c_uint32), ("queued", c_uint32), ("reserved", c_uint32),
                ("budget_bytes", c_uint64), ("held_bytes", c_uint64), ("busy_ms", c_double)]

    def as_dict(self) -> dict:
        return {k: (float(getattr(self, k)) if k == "busy_ms" else int(getattr(self, k)))
                for k, _ in self._fields_ if k != "reserved"}


class WgJobInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("phase", c_uint32), ("query", c_uint32), ("requeues", c_uint32),
                ("reservation_bytes", c_uint64), ("peak_bytes", c_uint64), ("submit_ms", c_double),
                ("start_ms", c_double), ("end_ms", c_double)]

    def as_dict(self) -> dict:
        return {k: (float(getattr(self, k)) if k.endswith("_ms") else int(getattr(self, k)))
                for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_uint64, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_uint64, c_void_p, c_void_p)


class WgAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


class WgError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_status_name(status)}: {detail}")
        self.status = status


_lib = None

# (name, restype, argtypes) of every exported entry point.
SIGNATURES = [
    ("wg_engine_create", c_int, [c_int, POINTER(c_void_p)]),
    ("wg_engine_create_ex", c_int, [c_int, POINTER(WgAllocator), POINTER(c_void_p)]),
    ("wg_engine_destroy", None, [c_void_p]),
    ("wg_tc", c_int, [c_void_p, c_void_p, c_void_p, c_uint64, POINTER(WgOptions), c_void_p,
                      POINTER(c_void_p), POINTER(WgStats)]),
    ("wg_sg", c_int, [c_void_p, c_void_p, c_void_p, c_uint64, POINTER(WgOptions), c_void_p,
                      POINTER(c_void_p), POINTER(WgStats)]),
    ("wg_tc_batch", c_int, [c_void_p, c_uint32, c_void_p, c_void_p, c_void_p, c_uint64,
                            POINTER(WgOptions), c_void_p, POINTER(c_void_p), POINTER(WgStats)]),
    ("wg_sg_batch", c_int, [c_void_p, c_uint32, c_void_p, c_void_p, c_void_p, c_uint64,
                            POINTER(WgOptions), c_void_p, POINTER(c_void_p), POINTER(WgStats)]),
    ("wg_triangles", c_int, [c_void_p, c_void_p, c_void_p, c_uint64, POINTER(WgOptions), c_void_p,
                             POINTER(c_uint64), POINTER(WgStats)]),
    ("wg_sort_keys", c_int, [c_void_p, c_void_p, c_void_p, c_uint64, c_uint32, c_uint32, POINTER(WgOptions),
                             c_void_p, POINTER(WgStats)]),
    ("wg_sort_keys_noalloc", c_int, [c_void_p, c_void_p, c_uint64, c_uint32, c_uint32, c_void_p]),
    ("wg_merge_keys", c_int, [c_void_p, c_void_p, c_uint64, c_void_p, c_uint64, c_void_p, c_uint32,
                              POINTER(WgOptions), c_void_p, POINTER(WgStats)]),
    ("wg_result_instances", c_uint32, [c_void_p]),
    ("wg_result_offsets", c_int, [c_void_p, c_void_p, c_uint64, c_void_p]),
    ("wg_get_sort_config", c_int, [c_void_p, c_uint32, POINTER(WgSortConfig)]),
    ("wg_set_sort_config", c_int, [c_void_p, c_uint32, POINTER(WgSortConfig)]),
    ("wg_autotune", c_int, [c_void_p, c_int, c_uint32, c_void_p, c_void_p, c_void_p, c_uint64,
                            POINTER(WgOptions), c_uint32, c_void_p, POINTER(WgTuneReport)]),
    ("wg_server_create", c_int, [c_int, POINTER(WgServerConfig), POINTER(c_void_p)]),
    ("wg_server_destroy", None, [c_void_p]),
    ("wg_submit", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_uint64, POINTER(WgOptions),
                          POINTER(c_void_p)]),
    ("wg_poll", c_int, [c_void_p, POINTER(c_int)]),
    ("wg_wait", c_int, [c_void_p, POINTER(c_void_p), POINTER(WgStats)]),
    ("wg_cancel", c_int, [c_void_p]),
    ("wg_job_get_info", c_int, [c_void_p, POINTER(WgJobInfo)]),
    ("wg_job_free", None, [c_void_p]),
    ("wg_server_get_stats", c_int, [c_void_p, POINTER(WgServerStats)]),
    ("wg_probe_sync_costs", c_int, [c_int, c_uint32, c_uint32, POINTER(c_double), POINTER(c_double),
                                    POINTER(c_double), POINTER(c_double)]),
    ("wg_result_size", c_uint64, [c_void_p]),
    ("wg_result_copy", c_int, [c_void_p, c_void_p, c_void_p, c_uint64, c_void_p]),
    ("wg_result_free", None, [c_void_p]),
    ("wg_status_string", c_char_p, [c_int]),
    ("wg_last_error", c_char_p, [c_void_p]),
]


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (run python -m paper_2607_17571_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _status_name(status: int) -> str:
    try:
        return lib().wg_status_string(status).decode()
    except Exception:  # noqa: BLE001 - only for messages
        return f"status {status}"


# ----------------------------------------------------------------------------
# Entry points with the C names (argument marshalling only).
# ----------------------------------------------------------------------------

def wg_engine_create(device: int = 0) -> c_void_p:
    eng = c_void_p()
    st = lib().wg_engine_create(device, byref(eng))
    if st != WG_OK:
        raise WgError(st, f"wg_engine_create(device={device})")
    return eng


def wg_engine_create_ex(device: int = 0, allocator: WgAllocator | None = None) -> c_void_p:
    eng = c_void_p()
    st = lib().wg_engine_create_ex(device, byref(allocator) if allocator is not None else None, byref(eng))
    if st != WG_OK:
        raise WgError(st, f"wg_engine_create_ex(device={device})")
    return eng


def wg_engine_destroy(engine) -> None:
    lib().wg_engine_destroy(engine)


def wg_tc(engine, d_src: int, d_dst: int, m: int, options: WgOptions | None, stream: int,
          stats: WgStats | None = None):
    """Returns (status, result handle)."""
    res = c_void_p()
    st = lib().wg_tc(engine, c_void_p(d_src), c_void_p(d_dst), m,
                     byref(options) if options is not None else None, c_void_p(stream),
                     byref(res), byref(stats) if stats is not None else None)
    return st, res


def wg_sg(engine, d_src: int, d_dst: int, m: int, options: WgOptions | None, stream: int,
          stats: WgStats | None = None):
    res = c_void_p()
    st = lib().wg_sg(engine, c_void_p(d_src), c_void_p(d_dst), m,
                     byref(options) if options is not None else None, c_void_p(stream),
                     byref(res), byref(stats) if stats is not None else None)
    return st, res


def _batch(fn, engine, num: int, d_offsets: int, d_src: int, d_dst: int, m: int,
           options: WgOptions | None, stream: int, stats: WgStats | None):
    res = c_void_p()
    st = fn(engine, num, c_void_p(d_offsets), c_void_p(d_src), c_void_p(d_dst), m,
            byref(options) if options is not None else None, c_void_p(stream), byref(res),
            byref(stats) if stats is not None else None)
    return st, res


def wg_tc_batch(engine, num: int, d_offsets: int, d_src: int, d_dst: int, m: int,
                options: WgOptions | None, stream: int, stats: WgStats | None = None):
    """Returns (status, result handle)."""
    return _batch(lib().wg_tc_batch, engine, num, d_offsets, d_src, d_dst, m, options, stream, stats)


def wg_sg_batch(engine, num: int, d_offsets: int, d_src: int, d_dst: int, m: int,
                options: WgOptions | None, stream: int, stats: WgStats | None = None):
    return _batch(lib().wg_sg_batch, engine, num, d_offsets, d_src, d_dst, m, options, stream, stats)


def wg_sort_keys(engine, d_keys: int, d_tmp: int, n: int, key_bytes: int, key_bits: int,
                 options: WgOptions | None, stream: int, stats: WgStats | None = None) -> int:
    return lib().wg_sort_keys(engine, c_void_p(d_keys), c_void_p(d_tmp), n, key_bytes, key_bits,
                              byref(options) if options is not None else None, c_void_p(stream),
                              byref(stats) if stats is not None else None)


def wg_sort_keys_noalloc(d_keys: int, d_tmp: int, n: int, key_bytes: int, key_bits: int, stream: int) -> int:
    return lib().wg_sort_keys_noalloc(c_void_p(d_keys), c_void_p(d_tmp), n, key_bytes, key_bits,
                                      c_void_p(stream))


def wg_probe_sync_costs(device: int, blocks: int, rounds: int) -> tuple:
    """wg_probe_sync_costs: microseconds per grid-wide barrier in one cooperative launch
    (flat, two-level, the runtime's grid sync) and per dependent launch of an empty kernel
    of the same shape."""
    bar, bar2, bcg, lau = c_double(0.0), c_double(0.0), c_double(0.0), c_double(0.0)
    st = lib().wg_probe_sync_costs(device, blocks, rounds, byref(bar), byref(bar2), byref(bcg), byref(lau))
    if st != WG_OK:
        raise WgError(st, "wg_probe_sync_costs")
    return bar.value, bar2.value, bcg.value, lau.value


def wg_merge_keys(engine, d_a: int, na: int, d_b: int, nb: int, d_out: int, key_bytes: int,
                  options: WgOptions | None, stream: int, stats: WgStats | None = None) -> int:
    return lib().wg_merge_keys(engine, c_void_p(d_a), na, c_void_p(d_b), nb, c_void_p(d_out), key_bytes,
                               byref(options) if options is not None else None, c_void_p(stream),
                               byref(stats) if stats is not None else None)


def wg_triangles(engine, d_src: int, d_dst: int, m: int, options: WgOptions | None, stream: int,
                 stats: WgStats | None = None):
    """Returns (status, count)."""
    count = c_uint64(0)
    st = lib().wg_triangles(engine, c_void_p(d_src), c_void_p(d_dst), m,
                            byref(options) if options is not None else None, c_void_p(stream),
                            byref(count), byref(stats) if stats is not None else None)
    return st, int(count.value)


def wg_result_instances(result) -> int:
    return int(lib().wg_result_instances(result))


def wg_result_offsets(result, offsets_out: int, capacity: int, stream: int) -> int:
    return lib().wg_result_offsets(result, c_void_p(offsets_out), capacity, c_void_p(stream))


def wg_get_sort_config(engine, key_bytes: int):
    cfg = WgSortConfig()
    st = lib().wg_get_sort_config(engine, key_bytes, byref(cfg))
    return st, cfg


def wg_set_sort_config(engine, key_bytes: int, cfg: WgSortConfig) -> int:
    return lib().wg_set_sort_config(engine, key_bytes, byref(cfg))


def wg_autotune(engine, query: int, num: int, d_offsets: int, d_src: int, d_dst: int, m: int,
                options: WgOptions | None, repeats: int, stream: int):
    """Returns (status, WgTuneReport)."""
    rep = WgTuneReport()
    st = lib().wg_autotune(engine, query, num, c_void_p(d_offsets), c_void_p(d_src), c_void_p(d_dst),
                           m, byref(options) if options is not None else None, repeats,
                           c_void_p(stream), byref(rep))
    return st, rep


def wg_server_create(device: int = 0, slots: int = 0, mem_budget_bytes: int = 0, hold_after_us: int = 0) -> c_void_p:
    srv = c_void_p()
    st = lib().wg_server_create(device, byref(WgServerConfig(slots, hold_after_us, mem_budget_bytes)), byref(srv))
    if st != WG_OK:
        raise WgError(st, f"wg_server_create(device={device})")
    return srv


def wg_server_destroy(server) -> None:
    lib().wg_server_destroy(server)


def wg_submit(server, query: int, src: int, dst: int, m: int, options: WgOptions | None):
    """Returns (status, job handle); src / dst are device or host addresses."""
    job = c_void_p()
    st = lib().wg_submit(server, query, c_void_p(src), c_void_p(dst), m,
                         byref(options) if options is not None else None, byref(job))
    return st, job


def wg_poll(job) -> tuple[int, bool]:
    done = c_int(0)
    st = lib().wg_poll(job, byref(done))
    return st, bool(done.value)


def wg_wait(job, stats: WgStats | None = None):
    """Returns (status, result handle or None)."""
    res = c_void_p()
    st = lib().wg_wait(job, byref(res), byref(stats) if stats is not None else None)
    return st, res


def wg_cancel(job) -> int:
    return lib().wg_cancel(job)


def wg_job_get_info(job) -> WgJobInfo:
    info = WgJobInfo()
    lib().wg_job_get_info(job, byref(info))
    return info


def wg_job_free(job) -> None:
    lib().wg_job_free(job)


def wg_server_get_stats(server) -> WgServerStats:
    out = WgServerStats()
    lib().wg_server_get_stats(server, byref(out))
    return out


def wg_result_size(result) -> int:
    return int(lib().wg_result_size(result))


def wg_result_copy(result, src_out: int, dst_out: int, capacity: int, stream: int) -> int:
    return lib().wg_result_copy(result, c_void_p(src_out), c_void_p(dst_out), capacity, c_void_p(stream))


def wg_result_free(result) -> None:
    lib().wg_result_free(result)


def wg_status_string(status: int) -> str:
    return lib().wg_status_string(status).decode()


def wg_last_error(engine) -> str:
    return lib().wg_last_error(engine).decode()


# ----------------------------------------------------------------------------
# torch conveniences
# ----------------------------------------------------------------------------

def make_options(flags: int = 0, batch_k: int = 0, loop_mode: int = WG_LOOP_AUTO,
                 radix_field_bits: int = 0, max_iterations: int = 0, mem_budget_bytes: int = 0,
                 force_overflow_at_iter: int = 0, timing_stages: int = 0,
                 radix_digit_bits: int = 0, tile_items: int = 0) -> WgOptions:
    o = WgOptions()
    o.struct_size = ctypes.sizeof(WgOptions)
    o.flags = flags
    o.batch_k = batch_k
    o.loop_mode = loop_mode
    o.radix_field_bits = radix_field_bits
    o.max_iterations = max_iterations
    o.mem_budget_bytes = mem_budget_bytes
    o.force_overflow_at_iter = force_overflow_at_iter
    o.timing_stages = timing_stages
    o.radix_digit_bits = radix_digit_bits
    o.tile_items = tile_items
    return o


def stats_dict(s: WgStats, deltas=None) -> dict:
    d = {
        "iterations": int(s.iterations), "result_tuples": int(s.result_tuples),
        "base_tuples": int(s.base_tuples), "join_candidates": int(s.join_candidates),
        "host_syncs": int(s.host_syncs), "resumes": int(s.resumes),
        "field_bits": int(s.field_bits), "key_bytes": int(s.key_bytes),
        "digit_bits": int(s.digit_bits), "sort_passes": int(s.sort_passes),
        "tail_iterations": int(s.tail_iterations), "solve_ms": float(s.solve_ms),
        "stage_ms": {k: float(s.stage_ms[i]) for i, k in enumerate(STAGES)},
        "stage_launches": {k: int(s.stage_launches[i]) for i, k in enumerate(STAGES)},
        "stage_bytes": {k: int(s.stage_bytes[i]) for i, k in enumerate(STAGES)},
    }
    if deltas is not None:
        d["delta_sizes"] = [int(deltas[i]) for i in range(min(int(s.iterations) + 1, len(deltas)))]
    return d


class TorchAllocator:
    """wg_allocator hooks that take the engine's device memory from torch's caching allocator.

    The C side calls them on the thread that called into the engine (with the GIL released
    by ctypes; the callbacks take it back).  A block is returned to torch on the stream it
    was allocated on; when the engine frees it after using it on another stream, that stream
    is drained first, since torch would otherwise reuse the block in the allocating stream's
    order only.  ``allocs`` / ``frees`` / ``live`` count the calls (for tests)."""

    def __init__(self, device: int = 0):
        self.device = device
        self.allocs = 0
        self.frees = 0
        self.failed = 0
        self.live = {}  # pointer -> (bytes, allocating stream)
        self._alloc = ALLOC_FN(self._on_alloc)
        self._free = FREE_FN(self._on_free)
        self.struct = WgAllocator(self._alloc, self._free, None)

    def _on_alloc(self, nbytes, stream, user):
        import torch

        try:
            s = int(stream or 0)
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, s)
        except Exception:  # noqa: BLE001 - reported to the engine as a failed allocation
            self.failed += 1
            return None
        self.allocs += 1
        self.live[int(p)] = (int(nbytes), s)
        return p

    def _on_free(self, ptr, nbytes, stream, user):
        import torch

        p = int(ptr or 0)
        if not p:
            return
        _, s_alloc = self.live.pop(p, (0, 0))
        if int(stream or 0) != s_alloc:
            torch.cuda.synchronize(self.device)
        torch.cuda.caching_allocator_delete(p)
        self.frees += 1


class Engine:
    """One engine per device and host thread; results stay valid until its next solve.

    ``allocator="torch"`` (or a TorchAllocator) routes every device allocation of the
    engine through torch's caching allocator (wg_engine_create_ex); None takes the
    library's stream-ordered default."""

    def __init__(self, device: int = 0, allocator=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the fixpoint engine needs a ROCm GPU")
        self.device = device
        if allocator == "torch":
            allocator = TorchAllocator(device)
        self.allocator = allocator  # kept alive: the C side holds its function pointers
        if allocator is None:
            self.handle = wg_engine_create(device)
        else:
            self.handle = wg_engine_create_ex(device, allocator.struct)

    def close(self):
        if self.handle is not None:
            wg_engine_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def solve(self, query: str, src, dst, options: WgOptions | None = None, max_deltas: int = 1 << 16,
              want_result: bool = True):
        """Run wg_tc / wg_sg on torch uint32/int32 CUDA tensors; returns (src, dst, stats)."""
        import torch

        src, dst, _ = self._check_edges(src, dst)
        stream = torch.cuda.current_stream(src.device).cuda_stream
        stats = WgStats()
        deltas = (c_uint64 * max_deltas)()
        stats.delta_sizes = deltas
        stats.delta_sizes_cap = max_deltas
        fn = wg_tc if query == "tc" else wg_sg
        st, res = fn(self.handle, src.data_ptr(), dst.data_ptr(), src.numel(), options, stream, stats)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        out_s, out_d, _ = self._take(res, src.device, stream, want_result, False)
        return out_s, out_d, stats_dict(stats, deltas)

    def _take(self, res, device, stream, want_result, want_offsets):
        """Copy a result handle into torch tensors (split arrays, optional offsets) and free it."""
        import torch

        try:
            n = wg_result_size(res)
            out_s = out_d = offs = None
            if want_result:
                out_s = torch.empty(n, dtype=torch.uint32, device=device)
                out_d = torch.empty(n, dtype=torch.uint32, device=device)
                if n:
                    st = wg_result_copy(res, out_s.data_ptr(), out_d.data_ptr(), n, stream)
                    if st != WG_OK:
                        raise WgError(st, wg_last_error(self.handle))
            if want_offsets:
                k = wg_result_instances(res)
                offs = torch.empty(k + 1, dtype=torch.int64, device=device)
                st = wg_result_offsets(res, offs.data_ptr(), k + 1, stream)
                if st != WG_OK:
                    raise WgError(st, wg_last_error(self.handle))
        finally:
            wg_result_free(res)
        return out_s, out_d, offs

    @staticmethod
    def _check_edges(src, dst, offsets=None):
        import torch

        if src.device.type != "cuda" or dst.device.type != "cuda":
            raise ValueError("edge tensors must live on the GPU")
        if src.shape != dst.shape or src.dim() != 1:
            raise ValueError("src and dst must be 1-D tensors of equal length")
        if src.dtype not in (torch.uint32, torch.int32) or dst.dtype != src.dtype:
            raise ValueError("edge tensors must be uint32 (or int32 bit patterns)")
        if offsets is not None:
            if offsets.device.type != "cuda" or offsets.dim() != 1 or offsets.numel() < 2:
                raise ValueError("offsets must be a 1-D GPU tensor of instances + 1 entries")
            if offsets.dtype not in (torch.int64, torch.uint64):
                raise ValueError("offsets must be int64 (or uint64)")
        return src.contiguous(), dst.contiguous(), None if offsets is None else offsets.contiguous()

    def solve_batch(self, query: str, src, dst, offsets, options: WgOptions | None = None,
                    want_result: bool = True, max_deltas: int = 1 << 16):
        """wg_tc_batch / wg_sg_batch; returns (src, dst, result offsets, stats)."""
        import torch

        src, dst, offsets = self._check_edges(src, dst, offsets)
        stream = torch.cuda.current_stream(src.device).cuda_stream
        stats = WgStats()
        deltas = (c_uint64 * max_deltas)()
        stats.delta_sizes = deltas
        stats.delta_sizes_cap = max_deltas
        fn = wg_tc_batch if query == "tc" else wg_sg_batch
        st, res = fn(self.handle, offsets.numel() - 1, offsets.data_ptr(), src.data_ptr(), dst.data_ptr(),
                     src.numel(), options, stream, stats)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        out_s, out_d, offs = self._take(res, src.device, stream, want_result, True)
        return out_s, out_d, offs, stats_dict(stats, deltas)

    def autotune(self, query: str, src, dst, offsets=None, options: WgOptions | None = None,
                 repeats: int = 2) -> dict:
        """wg_autotune on a single instance (offsets None) or a batch; returns the report."""
        import torch

        src, dst, offsets = self._check_edges(src, dst, offsets)
        stream = torch.cuda.current_stream(src.device).cuda_stream
        num = 0 if offsets is None else offsets.numel() - 1
        st, rep = wg_autotune(self.handle, WG_QUERY_TC if query == "tc" else WG_QUERY_SG, num,
                              0 if offsets is None else offsets.data_ptr(), src.data_ptr(),
                              dst.data_ptr(), src.numel(), options, repeats, stream)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        return rep.as_dict()

    def triangles(self, src, dst, options: WgOptions | None = None):
        """wg_triangles on torch uint32/int32 CUDA tensors; returns (count, stats)."""
        import torch

        src, dst, _ = self._check_edges(src, dst)
        stream = torch.cuda.current_stream(src.device).cuda_stream
        stats = WgStats()
        st, count = wg_triangles(self.handle, src.data_ptr(), dst.data_ptr(), src.numel(), options,
                                 stream, stats)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        return count, stats_dict(stats)

    @staticmethod
    def _check_keys(t, name: str):
        import torch

        if not t.is_cuda or t.dtype not in (torch.int32, torch.uint32, torch.int64, torch.uint64):
            raise ValueError(f"{name} must be a CUDA tensor of 32- or 64-bit integers")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t.element_size()

    def sort_keys(self, keys, tmp, key_bits: int, options: WgOptions | None = None):
        """wg_sort_keys: sorts `keys` (CUDA, 32- or 64-bit, read as unsigned) in place with the
        LSD passes; `tmp` is scratch of the same size and type.  Returns the stats."""
        import torch

        kb = self._check_keys(keys, "keys")
        if self._check_keys(tmp, "tmp") != kb or tmp.numel() < keys.numel():
            raise ValueError("tmp must match keys in type and hold as many keys")
        stream = torch.cuda.current_stream(keys.device).cuda_stream
        stats = WgStats()
        st = wg_sort_keys(self.handle, keys.data_ptr(), tmp.data_ptr(), keys.numel(), kb, key_bits,
                          options, stream, stats)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        return stats_dict(stats)

    def merge_keys(self, a, b, out, options: WgOptions | None = None):
        """wg_merge_keys: out = merge of the ascending runs a and b (CUDA, same integer type)."""
        import torch

        kb = self._check_keys(a, "a")
        if self._check_keys(b, "b") != kb or self._check_keys(out, "out") != kb:
            raise ValueError("a, b and out must have the same key width")
        if out.numel() < a.numel() + b.numel():
            raise ValueError("out must hold a.numel() + b.numel() keys")
        stream = torch.cuda.current_stream(a.device).cuda_stream
        stats = WgStats()
        st = wg_merge_keys(self.handle, a.data_ptr(), a.numel(), b.data_ptr(), b.numel(), out.data_ptr(), kb,
                           options, stream, stats)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        return stats_dict(stats)

    def sort_config(self, key_bytes: int) -> dict:
        st, cfg = wg_get_sort_config(self.handle, key_bytes)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))
        return cfg.as_dict()

    def set_sort_config(self, key_bytes: int, digit_bits: int, tile_items: int, blocks: int) -> None:
        cfg = WgSortConfig(digit_bits, tile_items, blocks, 0)
        st = wg_set_sort_config(self.handle, key_bytes, cfg)
        if st != WG_OK:
            raise WgError(st, wg_last_error(self.handle))

    def tc(self, src, dst, options=None, **kw):
        return self.solve("tc", src, dst, options, **kw)

    def sg(self, src, dst, options=None, **kw):
        return self.solve("sg", src, dst, options, **kw)


class Job:
    """A request submitted to a Server."""

    def __init__(self, server: "Server", handle):
        self.server = server
        self.handle = handle

    def done(self) -> bool:
        return wg_poll(self.handle)[1]

    def cancel(self) -> None:
        wg_cancel(self.handle)

    def info(self) -> dict:
        return wg_job_get_info(self.handle).as_dict()

    def wait(self, want_result: bool = True, max_deltas: int = 1 << 16):
        """Block until done; returns (src, dst, stats, info).  Raises WgError on failure."""
        import torch

        stats = WgStats()
        deltas = (c_uint64 * max_deltas)()
        stats.delta_sizes = deltas
        stats.delta_sizes_cap = max_deltas
        st, res = wg_wait(self.handle, stats)
        info = self.info()
        if st != WG_OK:
            raise WgError(st, "served request failed")
        device = torch.device("cuda", self.server.device)
        stream = torch.cuda.current_stream(device).cuda_stream
        try:
            n = wg_result_size(res)
            out_s = out_d = None
            if want_result:
                out_s = torch.empty(n, dtype=torch.uint32, device=device)
                out_d = torch.empty(n, dtype=torch.uint32, device=device)
                if n:
                    st = wg_result_copy(res, out_s.data_ptr(), out_d.data_ptr(), n, stream)
                    if st != WG_OK:
                        raise WgError(st, "result copy")
        finally:
            wg_result_free(res)
        return out_s, out_d, stats_dict(stats, deltas), info

    def close(self) -> None:
        if self.handle is not None:
            wg_job_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Server:
    """Continuous-batching request server (wg_server_*) on one device."""

    def __init__(self, device: int = 0, slots: int = 0, mem_budget_bytes: int = 0, hold_after_us: int = 0):
        """hold_after_us: a solve running this long holds back admissions until it ends
        (0: the server's default, 0xFFFFFFFF: never)."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the request server needs a ROCm GPU")
        self.device = device
        self.handle = wg_server_create(device, slots, mem_budget_bytes, hold_after_us)

    def submit(self, query: str, src, dst, options: WgOptions | None = None) -> Job:
        """src / dst: torch tensors (GPU or CPU) or numpy arrays of uint32 ids."""
        import numpy as np

        keep = []
        ptrs = []
        for a in (src, dst):
            if isinstance(a, np.ndarray):
                a = np.ascontiguousarray(a, dtype=np.uint32)
                keep.append(a)
                ptrs.append(a.ctypes.data)
            else:
                a = a.contiguous()
                keep.append(a)
                ptrs.append(a.data_ptr())
        m = len(keep[0])
        if len(keep[1]) != m:
            raise ValueError("src and dst differ in length")
        q = WG_QUERY_TC if query == "tc" else WG_QUERY_SG
        st, job = wg_submit(self.handle, q, ptrs[0], ptrs[1], m, options)
        if st != WG_OK:
            raise WgError(st, "wg_submit")
        return Job(self, job)

    def stats(self) -> dict:
        return wg_server_get_stats(self.handle).as_dict()

    def close(self) -> None:
        if self.handle is not None:
            wg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
