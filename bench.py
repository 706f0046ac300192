"""Benchmark: derived tuples/s of TC / SG fixpoints on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

A step is one whole solve through the C ABI (wg_tc / wg_sg, or wg_tc_batch /
wg_sg_batch for batched workloads): prepare (sort, dedup and index E), every
semi-naive iteration (join, sort, fused dedup + difference, merge, empty-delta test)
and the result unpacked into torch-allocated split arrays.  Inputs are resident in HBM
before the timed region.  The value is |fixpoint| per second of solve time.

Default workload: TC on an R-MAT graph of scale 15 (32,768 vertices), m = 29,491,
(a,b,c,d) = (0.57,0.19,0.19,0.05), seed 2.  R-MAT scale 22 with 3.8M edges has a
closure of ~3.9e11 tuples, which no single GPU can hold; scale 15 keeps the same skew
and degree with a closure of 4.99e7 tuples.

Every workload first runs the sort autotuner (wg_autotune: digit width, tile, grid) on
its own input, outside the timed region (--no-autotune skips it).  Batched workloads
(tc_batch_er_4096: 4,096 ER instances in one solve) then also time the plain path: the
same instances solved one at a time with wg_tc.

The JSON line also carries the roofline of the dominant kernel: its algorithmic bytes
(include/wg.h, wg_stats.stage_bytes) over the HIP-event time of its launches, taken in a
second run of the same K solves with events around that kernel only (events cost launch
overlap, so the throughput figure comes from the run without them), against 8 TB/s of
HBM; and the CPU oracle timed on the host (test infrastructure, used only for this
baseline), with the CPU model and core counts.  The oracle is single-threaded; a batch
also gets an all-core figure, its instances spread over worker processes.

The default run (no --workload) adds under "extra" the same measurement of the batched
workload (tc_batch_er_4096, 3 solves, with the plain one-by-one path) and of SG on
sg_er_500k, each with its own roofline and CPU baseline, and the served mix (120 requests,
2 slots) at 0.7x, 1.0x and 1.5x the plain path's capacity: p50/p99 latency and tuples/s of
the server and of the plain path, both measured under the same Poisson arrivals, with
every served result checked against the oracle's record.  CPU baselines run first,
before anything touches the GPU, because the all-core leg forks worker processes.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# kernels behind each timed stage kind (include/wg.h, WG_STAGE_*)
STAGE_KERNELS = {
    "join_count": "k_join_count", "join_emit": "k_join_emit",
    "radix_hist": "k_radix_count + k_radix_scan", "radix_pass": "k_radix_scatter",
    "dedup_diff": "k_compact_local + k_compact_gather", "merge": "k_merge",
    "prepare": "k_max_id, k_pack, k_index_*, k_unpack", "seg_sort": "k_seg_sort",
    "row_diff": "k_row_diff + k_row_gather", "tail_loop": "k_tail_loop",
}
WORKLOAD_TEXT = {
    "tc_rmat_s15": "TC, R-MAT scale 15 (n=32,768, m=29,491, a,b,c,d=0.57,0.19,0.19,0.05, seed 2); "
                   "stands in for R-MAT scale 22 whose ~3.9e11-tuple closure exceeds one GPU",
    "tc_rmat_s16": "TC, R-MAT scale 16 (n=65,536, m=58,982, a,b,c,d=0.57,0.19,0.19,0.05, seed 2)",
    "tc_rmat_s15_ids24": "TC, R-MAT scale 15 with ids scattered into [0, 2^22) (22-bit radix fields, 64-bit keys)",
    "tc_er_2000": "TC, directed ER n=2,000 m=1,900 seed 1",
    "sg_er_500k": "SG, directed ER n=500,000 m=450,000 seed 3",
    "tc_grid_100": "TC, 100x100 grid DAG (198 iterations)",
    "tc_batch_er_4096": "batched TC, 4,096 ER instances, n log-uniform in [256, 65,536], mean "
                        "out-degree uniform in [0.5, 0.95], seed 4, one solve",
    "tc_batch_er_256": "batched TC, 256 ER instances (same recipe), seed 6",
    "sg_batch_er_256": "batched SG, 256 ER instances, n log-uniform in [64, 4,096], seed 7",
    "served_mix": "served TC/SG mix: Poisson arrivals at 0.7x the single-stream capacity, 70% TC / "
                  "30% SG, 50/50 ER / R-MAT(0.57,0.19,0.19,0.05), n log-uniform in [1k, 1M] (R-MAT "
                  "capped at scale 15), mean out-degree uniform in [0.5, 0.95], seed 5",
}


def kernel_source_digest() -> str:
    """sha256 of the kernel source: a stored HBM-traffic figure applies only to the kernels
    it was measured on."""
    import hashlib

    with open(os.path.join(ROOT, "paper_2607_17571_amd", "csrc", "wg_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, workload: str, digit_bits: int, tile_items: int):
    """Calibrated HBM bytes per launch of `kernel` on `workload` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs stored under profiles/ (null when none matches the current kernels and
    sort configuration)."""
    prof = os.path.join(ROOT, "profiles")
    if not os.path.isdir(prof):
        return None
    digest = kernel_source_digest()
    for name in sorted(os.listdir(prof)):
        if not name.endswith("_traffic.json"):
            continue
        with open(os.path.join(prof, name)) as f:
            rec = json.load(f)
        # the sort's digit width and tile matter only to the sort's own kernels
        sort_kernel = "k_radix" in kernel
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("kernel_source_sha256") == digest
                and (not sort_kernel or (rec.get("digit_bits") == digit_bits
                                         and rec.get("tile_items") == tile_items))):
            return rec
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default=None,
                   help="workload name (default tc_rmat_s15, with the batched and SG extras)")
    p.add_argument("--no-extras", action="store_true",
                   help="default run: skip the batched and SG measurements beside the headline")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-timing", action="store_true", help="time steps without per-kernel events")
    p.add_argument("--digit-bits", type=int, default=0, help="radix digit bits (0: engine's choice)")
    p.add_argument("--tile-items", type=int, default=0, help="sort tile keys per thread (0: engine's)")
    p.add_argument("--field-bits", type=int, default=0, help="radix field width per id (0: engine's)")
    p.add_argument("--no-autotune", action="store_true", help="skip the sort autotuner (run before timing)")
    p.add_argument("--no-plain", action="store_true", help="batched workloads: skip the one-by-one path")
    p.add_argument("--no-spec", action="store_true", help="no speculative batch behind host checks")
    p.add_argument("--no-tail-loop", action="store_true", help="no one-block tail loop (every iteration multi-block)")
    p.add_argument("--dominant", default=None, help="kernel kind to take the roofline of (skips the probe)")
    p.add_argument("--roofline-only", action="store_true",
                   help="run only the instrumented steps (value then comes from them); for profiling")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only copy MIB MiB device to device 10 times (counter calibration) and exit")
    p.add_argument("--gather-calibration", type=int, default=0, metavar="MIB",
                   help="only gather MIB MiB of 4-byte values through a random permutation 10 times "
                        "(scattered-read counter calibration) and exit")
    p.add_argument("--requests", type=int, default=120, help="served_mix: number of requests")
    p.add_argument("--slots", type=int, default=2,
                   help="served_mix: concurrent solves (2 measured ahead of 3 and 4 on this mix)")
    p.add_argument("--load", type=float, default=0.7, help="served_mix: offered load / capacity")
    p.add_argument("--hold-after-us", type=int, default=0,
                   help="served_mix: long-solve hold of the server (0: its default, 4294967295: never)")
    p.add_argument("--sync-probe", action="store_true",
                   help="cost of a grid-wide barrier in one cooperative launch against a dependent launch")
    p.add_argument("--kernel-sweep", action="store_true",
                   help="sort and merge kernels alone on 2^20..2^28 synthetic keys")
    p.add_argument("--sweep-min-log2", type=int, default=20)
    p.add_argument("--sweep-max-log2", type=int, default=28)
    p.add_argument("--ablation", choices=["join", "triangles", "sync", "engineering"], default=None,
                   help="time the variants of one design choice instead of the headline line")
    p.add_argument("--ablation-workloads", default=None,
                   help="comma-separated workload names for --ablation (default: per ablation)")
    a = p.parse_args()
    a.workload_given = a.workload is not None
    if a.workload is None:
        a.workload = "tc_rmat_s15"
    return a


SG_EXTRA = "sg_er_500k"
BATCH_EXTRA = "tc_batch_er_4096"


def is_batch(name: str) -> bool:
    return "_batch_" in name


def cpu_info() -> dict:
    """The host the CPU baseline ran on: CPU model, logical CPUs, and those this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


_POOL_BATCH = None  # (query, Batch) of the all-core leg, set before the workers fork


def _oracle_chunk(lo: int, hi: int):
    import oracle

    query, b = _POOL_BATCH
    fn = oracle.tc if query == "tc" else oracle.sg
    return sum(int(fn(*b.instance(i)).src.size) for i in range(lo, hi))


def _all_core(name: str, seconds: float = 15.0, max_workers: int = 16):
    """The unchanged oracle over a batch's instances in worker processes (one instance at a
    time per worker, chunks of 8 handed out in order until `seconds` have passed)."""
    import multiprocessing
    from concurrent.futures import FIRST_COMPLETED, ProcessPoolExecutor, wait

    from paper_2607_17571_amd import inputs

    global _POOL_BATCH
    _POOL_BATCH = inputs.batch_workload(name)
    num = _POOL_BATCH[1].num
    workers = max(1, min(cpu_info()["usable_cpus"] or 1, max_workers))
    chunk = 8
    with ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("fork")) as ex:
        list(ex.map(time.sleep, [0.05] * (2 * workers)))  # every worker started before the clock
        t0 = time.perf_counter()
        nxt = 0
        pending = set()
        tuples = 0
        while nxt < num and len(pending) < 2 * workers:
            pending.add(ex.submit(_oracle_chunk, nxt, min(nxt + chunk, num)))
            nxt = min(nxt + chunk, num)
        while pending:
            done, pending = wait(pending, return_when=FIRST_COMPLETED)
            tuples += sum(f.result() for f in done)
            for _ in done:
                if nxt < num and time.perf_counter() - t0 < seconds:
                    pending.add(ex.submit(_oracle_chunk, nxt, min(nxt + chunk, num)))
                    nxt = min(nxt + chunk, num)
        dt = time.perf_counter() - t0
    _POOL_BATCH = None
    return {"value": tuples / dt, "unit": "tuples/s", "cores": workers, "kind": "oracle",
            "sample": f"instances 0..{nxt - 1} of {name} ({tuples} tuples) in {dt:.2f} s over {workers} "
                      f"worker processes, each running the single-threaded oracle on one instance at a time"}


def cpu_baseline(name: str, all_core: bool = False):
    """The oracle as it stands, timed on the host: one whole solve, or for a batch the
    instances in order until about 15 s of work.  The oracle is plain single-threaded numpy
    (nothing in it is parallel); for a batch, `all_core` adds the same oracle over the
    instances in worker processes."""
    import oracle
    from paper_2607_17571_amd import inputs

    host = cpu_info()
    if is_batch(name):
        query, b = inputs.batch_workload(name)
        fn = oracle.tc if query == "tc" else oracle.sg
        t0 = time.perf_counter()
        tuples = done = 0
        while done < b.num and time.perf_counter() - t0 < 15.0:
            tuples += fn(*b.instance(done)).src.size
            done += 1
        dt = time.perf_counter() - t0
        out = {"value": tuples / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
               "sample": f"instances 0..{done - 1} of {name} ({tuples} tuples) solved one by one "
                         f"in {dt:.2f} s, single-threaded numpy", **host}
        if all_core:
            out["all_core"] = _all_core(name)
        return out, None
    w = inputs.workload(name)
    t0 = time.perf_counter()
    r = oracle.tc(w.src, w.dst) if w.query == "tc" else oracle.sg(w.src, w.dst)
    dt = time.perf_counter() - t0
    return {"value": r.src.size / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of {name} ({r.src.size} tuples, {r.iterations} iterations) "
                      f"in {dt:.2f} s, single-threaded numpy (one solve has no natural split)",
            **host}, r


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else 0.0


def served_cpu_baseline(reqs):
    import oracle

    t0 = time.perf_counter()
    tuples = done = 0
    while done < len(reqs) and time.perf_counter() - t0 < 15.0:
        r = reqs[done]
        tuples += (oracle.tc(r.src, r.dst) if r.query == "tc" else oracle.sg(r.src, r.dst)).src.size
        done += 1
    dt = time.perf_counter() - t0
    return {"value": tuples / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"requests 0..{done - 1} of the served mix ({tuples} tuples) solved one by "
                      f"one in {dt:.2f} s, single-threaded numpy"}


def run_kernel_sweep(args):
    """Single stages on synthetic keys of 2^20..2^28 elements (uniform random 30-bit keys in
    32-bit words, 48-bit keys in 64-bit words): the LSD sort's count (+ scan) and scatter
    kinds, and the merge of two sorted halves, each as algorithmic bytes over its kernel
    time (HIP events on the launches), best of 3 runs."""
    import torch

    from paper_2607_17571_amd import wg

    eng = wg.Engine(0)
    timing = wg.make_options(flags=wg.WG_STAGE_TIMING)
    rows = []
    for kb, bits in ((4, 30), (8, 48)):
        dt = torch.int32 if kb == 4 else torch.int64
        for lg in range(args.sweep_min_log2, args.sweep_max_log2 + 1):
            n = 1 << lg
            g = torch.Generator(device="cuda").manual_seed(lg * 10 + kb)
            src = torch.randint(0, 1 << bits, (n,), generator=g, device="cuda", dtype=torch.int64).to(dt)
            keys = torch.empty_like(src)
            tmp = torch.empty_like(src)
            best = {}
            for _ in range(3):
                keys.copy_(src)
                st = eng.sort_keys(keys, tmp, bits, timing)
                for k in ("radix_hist", "radix_pass"):
                    gbs = st["stage_bytes"][k] / (st["stage_ms"][k] * 1e6)
                    best[k] = max(best.get(k, 0.0), gbs)
            passes = st["sort_passes"]
            a, _ = torch.sort(src[: n // 2])
            b, _ = torch.sort(src[n // 2:])
            out = torch.empty_like(src)
            mg = 0.0
            for _ in range(3):
                st = eng.merge_keys(a, b, out, timing)
                mg = max(mg, st["stage_bytes"]["merge"] / (st["stage_ms"]["merge"] * 1e6))
            row = {"key_bytes": kb, "key_bits": bits, "n": n, "passes": passes,
                   "count_gbs": round(best["radix_hist"], 1),
                   "count_frac": round(best["radix_hist"] / HBM_PEAK_GBS, 4),
                   "scatter_gbs": round(best["radix_pass"], 1),
                   "scatter_frac": round(best["radix_pass"] / HBM_PEAK_GBS, 4),
                   "merge_gbs": round(mg, 1), "merge_frac": round(mg / HBM_PEAK_GBS, 4)}
            rows.append(row)
            _progress(f"sweep {kb * 8}-bit n=2^{lg}: count {row['count_frac']}, scatter "
                      f"{row['scatter_frac']}, merge {row['merge_frac']} of 8 TB/s")
            del src, keys, tmp, a, b, out
    cfg = {"4": eng.sort_config(4), "8": eng.sort_config(8)}
    eng.close()
    print(json.dumps({"kernel_sweep": rows, "peak_gbs": HBM_PEAK_GBS, "sort_config": cfg}), flush=True)


def _golden_served():
    """Per-request records of the served mix (size, iterations, sha256 of the lex-sorted
    pairs), written from the oracle by tests/golden/make_golden.py."""
    path = os.path.join(ROOT, "tests", "golden", "fixpoints.json")
    with open(path) as f:
        return json.load(f)["served_mix_120_seed5"]["requests"]


def _pairs_sha(s, d) -> str:
    import hashlib

    import numpy as np

    return hashlib.sha256(np.ascontiguousarray(s.cpu().numpy(), dtype="<u4").tobytes() +
                          np.ascontiguousarray(d.cpu().numpy(), dtype="<u4").tobytes()).hexdigest()


def measure_served(args):
    """The served mix under Poisson arrivals at 0.7x, 1.0x and 1.5x the plain path's capacity:
    continuous batching on the server against the plain path (one engine, one request at a
    time in arrival order), both measured under the same arrivals.  Every served result is
    checked against the oracle's record: size and iterations at every load, the sha256 of
    the pairs at the first load."""
    import numpy as np
    import torch

    from paper_2607_17571_amd import inputs, wg

    def progress(msg):
        print(f"[served] {msg}", file=sys.stderr, flush=True)

    reqs = inputs.served_requests(args.requests, seed=5)
    golden = _golden_served() if args.requests == 120 else None
    dev = [(torch.from_numpy(r.src).cuda(), torch.from_numpy(r.dst).cuda()) for r in reqs]
    torch.cuda.synchronize()
    progress(f"{len(reqs)} requests staged on the device")
    # the plain path's service times, back to back (they set the offered rates)
    eng = wg.Engine(0)
    for (s, d), r in list(zip(dev, reqs))[:4]:
        eng.solve(r.query, s, d, None)
    service, plain_tuples = [], 0
    for (s, d), r in zip(dev, reqs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, st = eng.solve(r.query, s, d, None, want_result=False)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t)
        plain_tuples += st["result_tuples"]
    capacity = len(reqs) / sum(service)
    progress(f"plain path: capacity {capacity:.1f} req/s ({sum(service):.2f} s of service)")
    srv = wg.Server(0, slots=args.slots, hold_after_us=getattr(args, "hold_after_us", 0))
    # warm-up as for the plain path, whose engine has solved every request once (the
    # service pass above) before its timed runs: the whole mix once through the server, so
    # that each slot's buffers have grown to what the mix needs
    warm = [srv.submit(r.query, s, d) for (s, d), r in zip(dev, reqs)]
    for job in warm:
        job.wait(want_result=False)
        job.close()
    progress("server warm")
    checks = {"size_iterations": 0, "sha256": 0, "mismatches": 0}

    def arrivals_at(load):
        rng = np.random.default_rng(5)
        gaps = rng.exponential(1.0 / (load * capacity), size=len(reqs))
        return np.cumsum(gaps) - gaps[0]

    def plain_at(arrivals):
        # one engine, requests in arrival order, each started when it has arrived and the
        # previous one is done (a FIFO queue in front of the plain path)
        lat, tuples = [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (s, d), r, a in zip(dev, reqs, arrivals):
            delay = t0 + a - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            _, _, st = eng.solve(r.query, s, d, None, want_result=False)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0 - a)
            tuples += st["result_tuples"]
        span = time.perf_counter() - t0
        return lat, tuples, span

    def served_at(arrivals, hash_results):
        jobs = []
        t0 = time.perf_counter()
        for (s, d), r, a in zip(dev, reqs, arrivals):
            delay = t0 + a - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            jobs.append(srv.submit(r.query, s, d))
        lat, tuples, first, last = [], 0, None, None
        for i, j in enumerate(jobs):
            s_, d_, st, info = j.wait(want_result=hash_results)
            lat.append((info["end_ms"] - info["submit_ms"]) / 1e3)
            tuples += st["result_tuples"]
            first = info["submit_ms"] if first is None else min(first, info["submit_ms"])
            last = info["end_ms"] if last is None else max(last, info["end_ms"])
            j.close()
            if golden is not None:
                rec = golden[i]
                checks["size_iterations"] += 1
                if st["result_tuples"] != rec["size"] or st["iterations"] != rec["iterations"]:
                    checks["mismatches"] += 1
                if hash_results:
                    checks["sha256"] += 1
                    if _pairs_sha(s_, d_) != rec["sha256"]:
                        checks["mismatches"] += 1
            del s_, d_
        return lat, tuples, (last - first) / 1e3

    sweep = []
    loads = sorted(set([args.load, 0.7, 1.0, 1.5]))
    for k, load in enumerate(loads):
        arr = arrivals_at(load)
        lat, tuples, span = served_at(arr, hash_results=(k == 0))
        plat, ptuples, pspan = plain_at(arr)
        res = {"load": load, "offered_req_per_s": round(load * capacity, 2),
               "served": {"p50_ms": round(1e3 * percentile(lat, 50), 3),
                          "p99_ms": round(1e3 * percentile(lat, 99), 3),
                          "tuples_per_s": round(tuples / span, 1), "span_ms": round(1e3 * span, 3)},
               "single_instance_path": {"p50_ms": round(1e3 * percentile(plat, 50), 3),
                                        "p99_ms": round(1e3 * percentile(plat, 99), 3),
                                        "tuples_per_s": round(ptuples / pspan, 1), "span_ms": round(1e3 * pspan, 3),
                                        "measured": True}}
        progress(f"load {load}: {res}")
        sweep.append(res)
    eng.close()
    stats = srv.stats()
    srv.close()
    head = next(x for x in sweep if x["load"] == args.load)
    return {
        "metric": "derived tuples/sec per TC/SG fixpoint; p50/p99 served latency",
        "value": head["served"]["tuples_per_s"],
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": len(reqs),
        "ms_per_step": head["served"]["span_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["served_mix"], "name": "served_mix",
                   "requests": len(reqs), "slots": args.slots, "edges": int(sum(len(r.src) for r in reqs)),
                   "tc_requests": sum(r.query == "tc" for r in reqs),
                   "offered_rate_per_s": head["offered_req_per_s"], "load": args.load},
        "served": dict(head["served"], max_running=stats["max_running"], requeued=stats["requeued"],
                       failed=stats["failed"]),
        "single_instance_path": dict(head["single_instance_path"],
                                     capacity_req_per_s=round(capacity, 2),
                                     service_ms_p50=round(1e3 * percentile(service, 50), 3),
                                     service_ms_max=round(1e3 * max(service), 3)),
        "load_sweep": sweep,
        "golden_checks": checks if golden is not None else None,
        "roofline": None,
    }


def run_served(args):
    """Continuous batching under Poisson arrivals vs the plain one-at-a-time path."""
    import torch  # noqa: F401

    from paper_2607_17571_amd import inputs

    cb = None
    if not args.no_cpu_baseline:
        cb = served_cpu_baseline(inputs.served_requests(args.requests, seed=5))
    out = measure_served(args)
    out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# Ablations: the same solves with one design choice switched, each variant timed over
# the same K steps after W warmup solves (no events in the timed solves; one extra solve
# with events on every kernel gives the per-stage split).  One JSON line per ablation.
# ---------------------------------------------------------------------------
ABLATION_DEFAULTS = {
    "join": "tc_rmat_s15,tc_rmat_s16",
    "triangles": "tri_rmat_s14,tri_rmat_s16",
    "sync": "tc_er_2000,sg_er_500k,tc_grid_100",
    "engineering": "tc_rmat_s15,sg_er_500k,tc_er_2000,tc_grid_100",
}
TRIANGLE_GRAPHS = {  # R-MAT stand-ins for SNAP graphs with hubs of out-degree in the thousands
    "tri_rmat_s14": (14, 8 << 14), "tri_rmat_s16": (16, 8 << 16), "tri_rmat_s17": (17, 8 << 17),
}


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _time_variant(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        st = fn(False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    probe = fn(True)
    return ms, st, probe


def _latencies(torch):
    """Host round-trip latencies of the runtime: the cost the loop policies trade."""
    reps = 2000
    x = torch.zeros(1, dtype=torch.int32, device="cuda")
    h = torch.empty(1, dtype=torch.int32, pin_memory=True)
    s = torch.cuda.current_stream()
    out = {}

    def clock(name, body):
        for _ in range(50):
            body()
        t0 = time.perf_counter()
        for _ in range(reps):
            body()
        out[name] = round(1e6 * (time.perf_counter() - t0) / reps, 2)

    clock("sync_idle_stream_us", lambda: s.synchronize())
    ev = torch.cuda.Event()

    def fence():
        ev.record(s)
        ev.synchronize()
    clock("event_record_wait_us", fence)

    def readback():
        h.copy_(x, non_blocking=True)
        s.synchronize()
    clock("readback_4B_us", readback)

    def launch_wait():
        x.add_(1)
        s.synchronize()
    clock("kernel_launch_wait_us", launch_wait)

    def launches():
        x.add_(1)
    clock("kernel_launch_enqueue_us", launches)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(s)
    with torch.cuda.stream(cs):
        x.add_(1)
        cs.synchronize()
        with torch.cuda.graph(g, stream=cs):
            for _ in range(32):
                x.add_(1)
    s.wait_stream(cs)
    s.synchronize()

    def graph_wait():
        g.replay()
        torch.cuda.current_stream().synchronize()
    clock("graph_32_kernels_replay_wait_us", graph_wait)

    def eager_wait():
        for _ in range(32):
            x.add_(1)
        s.synchronize()
    clock("eager_32_kernels_wait_us", eager_wait)
    return out


def run_ablation(args):
    import numpy as np  # noqa: F401
    import torch

    from paper_2607_17571_amd import inputs, wg

    names = (args.ablation_workloads or ABLATION_DEFAULTS[args.ablation]).split(",")
    eng = wg.Engine(0)
    T = wg.WG_STAGE_TIMING
    results = {}
    extra = {}
    for name in names:
        if args.ablation == "triangles":
            scale, m = TRIANGLE_GRAPHS[name]
            s_np, d_np = inputs.rmat(scale, m, *inputs.RMAT_ABCD, seed=scale)
            src, dst = torch.from_numpy(s_np).cuda(), torch.from_numpy(d_np).cuda()
            variants = {"sorted": 0, "hash": wg.WG_JOIN_HASH, "hash_rows": wg.WG_JOIN_HASH_ROWS}
            row = {"graph": f"R-MAT scale {scale}, m={len(s_np)}, seed {scale}",
                   "max_out_degree": int(np.bincount(s_np).max())}
            for vname, fl in variants.items():
                def fn(timing, fl=fl):
                    return eng.triangles(src, dst, wg.make_options(flags=fl | (T if timing else 0)))
                ms, (count, st), (_, pr) = _time_variant(torch, fn, args.steps, args.warmup)
                row[vname] = {"ms": round(ms, 3), "triangles": count,
                              "two_paths": st["join_candidates"],
                              "join_ms": round(pr["stage_ms"]["join_count"] + pr["stage_ms"]["join_emit"], 3),
                              "prepare_ms": round(pr["stage_ms"]["prepare"], 3)}
                _progress(f"{name} {vname}: {row[vname]}")
            row["triangles_per_edge"] = round(row["sorted"]["triangles"] / max(1, len(s_np)), 2)
            row["hash_over_sorted"] = round(row["hash"]["ms"] / row["sorted"]["ms"], 3)
            row["hash_rows_over_sorted"] = round(row["hash_rows"]["ms"] / row["sorted"]["ms"], 3)
            row["agree"] = all(row[v]["triangles"] == row["sorted"]["triangles"] for v in variants)
            results[name] = row
            continue
        w = inputs.workload(name)
        src, dst = torch.from_numpy(w.src).cuda(), torch.from_numpy(w.dst).cuda()
        if args.ablation == "join":
            variants = {"sorted": {}, "hash": dict(flags=wg.WG_JOIN_HASH),
                        "hash_rows": dict(flags=wg.WG_JOIN_HASH_ROWS)}
        elif args.ablation == "sync":
            ns = wg.WG_NO_SPECULATION
            variants = {
                "per_stage_readback": dict(loop_mode=wg.WG_LOOP_STAGE),
                "per_iteration_readback": dict(loop_mode=wg.WG_LOOP_HOST, flags=ns),
                "batch_10": dict(loop_mode=wg.WG_LOOP_BATCHED, batch_k=10, flags=ns),
                "batch_30": dict(loop_mode=wg.WG_LOOP_BATCHED, batch_k=30, flags=ns),
                "paper_adaptive": dict(loop_mode=wg.WG_LOOP_BATCHED, flags=ns),
                "paper_adaptive_speculative": dict(loop_mode=wg.WG_LOOP_BATCHED),
                "default": {},
                "default_graph_replay": dict(flags=wg.WG_ITER_GRAPH),
                "no_tail_loop": dict(flags=wg.WG_NO_TAIL_LOOP),
            }
            if w.query == "tc":
                for k in (2, 5, 20, 40, 50):
                    variants[f"batch_{k}"] = dict(loop_mode=wg.WG_LOOP_BATCHED, batch_k=k, flags=ns)
            for k in (1, 2, 4, 8, 16):
                variants[f"batch_{k}_speculative"] = dict(loop_mode=wg.WG_LOOP_BATCHED, batch_k=k)
        else:
            # the paper's adaptive width rounds the largest id's bit length up to 16, 24 or 32
            mx = int(max(w.src.max(), w.dst.max())) if w.src.size else 0
            paper_w = 16 if mx < (1 << 16) else (24 if mx < (1 << 24) else 32)
            variants = {
                "default": {},
                "unfused_dedup_diff": dict(flags=wg.WG_UNFUSED_DEDUP),
                "lsd_sort_only": dict(flags=wg.WG_LSD_SORT),
                "digits_8_exact_width": dict(radix_digit_bits=8),
                "digits_8_width_16_24_32": dict(radix_digit_bits=8, radix_field_bits=paper_w),
                "digits_8_fixed_32bit_fields": dict(radix_digit_bits=8, radix_field_bits=32),
            }
        row = {"query": w.query, "edges": int(w.src.size)}
        tuples = None
        for vname, kw in variants.items():
            kw = dict(kw)
            fl = kw.pop("flags", 0)

            def fn(timing, fl=fl, kw=kw):
                return eng.solve(w.query, src, dst, wg.make_options(flags=fl | (T if timing else 0), **kw),
                                 )[2]
            ms, st, pr = _time_variant(torch, fn, args.steps, args.warmup)
            if tuples is None:
                tuples = st["result_tuples"]
            elif st["result_tuples"] != tuples:
                raise SystemExit(f"{name} {vname}: {st['result_tuples']} tuples, expected {tuples}")
            row[vname] = {"ms_per_step": round(ms, 3), "host_syncs": st["host_syncs"],
                          "iterations": st["iterations"], "tail_iterations": st["tail_iterations"],
                          "sort_passes": st["sort_passes"],
                          "stage_ms": {k: round(v, 3) for k, v in pr["stage_ms"].items()}}
            _progress(f"{name} {vname}: {ms:.3f} ms, {st['host_syncs']} host syncs")
        row["fixpoint_tuples"] = tuples
        results[name] = row
    if args.ablation == "sync":
        extra["latency"] = _latencies(torch)
        _progress(f"latencies: {extra['latency']}")
    eng.close()
    out = {"ablation": args.ablation, "steps": args.steps, "warmup": args.warmup, "n_gpus": 1,
           "data": "synthetic", "results": results}
    out.update(extra)
    print(json.dumps(out), flush=True)


def measure(args, name: str) -> dict:
    """K timed solves of one workload (after the autotuner and W warm-ups), then the same K
    with events on the dominant kernel kind: the bench line without its CPU baseline."""
    import numpy as np
    import torch

    from paper_2607_17571_amd import inputs, wg

    eng = wg.Engine(0)
    extra = {}
    if is_batch(name):
        query, b = inputs.batch_workload(name)
        src = torch.from_numpy(b.src).cuda()
        dst = torch.from_numpy(b.dst).cuda()
        offs = torch.from_numpy(b.offsets.astype(np.int64)).cuda()
        edges = int(b.src.size)
        if not args.no_autotune and not (args.digit_bits or args.tile_items):
            rep = eng.autotune(query, src, dst, offs)
            extra["autotune"] = {"best": rep["best"], "best_ms": round(rep["best_ms"], 3),
                                 "default_ms": round(rep["before_ms"], 3),
                                 "trials": len(rep["trials"])}

        def solve(opts):
            _, _, _, st = eng.solve_batch(query, src, dst, offs, opts)
            return st
    else:
        w = inputs.workload(name)
        query = w.query
        src = torch.from_numpy(w.src).cuda()
        dst = torch.from_numpy(w.dst).cuda()
        edges = int(w.src.size)
        if not args.no_autotune and not (args.digit_bits or args.tile_items or args.field_bits):
            # one-time sort tuning on this graph, outside the timed region (as for batches)
            rep = eng.autotune(query, src, dst, None)
            extra["autotune"] = {"best": rep["best"], "best_ms": round(rep["best_ms"], 3),
                                 "default_ms": round(rep["before_ms"], 3),
                                 "trials": len(rep["trials"])}

        def solve(opts):
            _, _, st = eng.solve(query, src, dst, opts)
            return st

    sort_opts = dict(radix_digit_bits=args.digit_bits, tile_items=args.tile_items,
                     radix_field_bits=args.field_bits)
    base_flags = (wg.WG_NO_SPECULATION if args.no_spec else 0) | (wg.WG_NO_TAIL_LOOP if args.no_tail_loop else 0)
    for _ in range(args.warmup):
        solve(wg.make_options(flags=base_flags, **sort_opts))
    torch.cuda.synchronize()
    # Untimed probe with events on every kernel kind: per-stage breakdown and the dominant
    # kernel kind, which the instrumented run after the timed region measures alone.
    if args.dominant:
        if args.dominant not in wg.STAGES:
            raise SystemExit(f"--dominant must be one of {wg.STAGES}")
        dom, probe_ms, probe_gb, probe_frac = args.dominant, None, None, None
    else:
        probe = solve(wg.make_options(flags=wg.WG_STAGE_TIMING | base_flags, **sort_opts))
        dom = max(wg.STAGES, key=lambda k: probe["stage_ms"][k])
        probe_ms = {k: round(v, 3) for k, v in probe["stage_ms"].items()}
        probe_gb = {k: round(v / 1e9, 4) for k, v in probe["stage_bytes"].items()}
        # every kernel kind against the HBM peak (algorithmic bytes / event time, one solve
        # with events on every launch, so slightly pessimistic for the small kinds)
        probe_frac = {k: round(probe["stage_bytes"][k] / (probe["stage_ms"][k] * 1e6) / HBM_PEAK_GBS, 4)
                      for k in probe["stage_ms"] if probe["stage_ms"][k] > 0}
    tuples = 0
    st = None
    ms_per_step = value = None
    if not args.roofline_only:
        # timed region: K whole solves, no instrumentation
        clean = wg.make_options(flags=base_flags, **sort_opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st = solve(clean)
            tuples += st["result_tuples"]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ms_per_step = 1e3 * elapsed / args.steps
        value = tuples / elapsed

    roofline = None
    if not args.no_timing:
        # the same K solves with HIP events stamped by the dispatches of the dominant kernel
        # kind only (hipExtLaunchKernelGGL on the engine's stream); the stamping slows
        # those kernels slightly, so the throughput comes from the run above
        timed = wg.make_options(flags=wg.WG_STAGE_TIMING | base_flags,
                                timing_stages=1 << wg.STAGES.index(dom), **sort_opts)
        ms = nbytes = launches = inst_tuples = 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            sti = solve(timed)
            ms += sti["stage_ms"][dom]
            nbytes += sti["stage_bytes"][dom]
            launches += sti["stage_launches"][dom]
            inst_tuples += sti["result_tuples"]
            st = sti if st is None else st
        torch.cuda.synchronize()
        inst_elapsed = time.perf_counter() - t1
        inst_ms = 1e3 * inst_elapsed / args.steps
        if value is None:
            ms_per_step, value = inst_ms, inst_tuples / inst_elapsed
        achieved = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        tile = args.tile_items or (extra["autotune"]["best"]["tile_items"] if "autotune" in extra
                                   else eng.sort_config(st["key_bytes"])["tile_items"])
        tr = measured_traffic(STAGE_KERNELS[dom], name, st["digit_bits"], tile)
        roofline = {"bound": "hbm", "kernel": STAGE_KERNELS[dom], "stage": dom,
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": tr["traffic_bytes_per_launch"] if tr else None,
                    "avg_launch_us": round(1e3 * ms / max(1, launches), 2),
                    "bytes_per_launch": nbytes // max(1, launches),
                    "launches_per_step": launches // args.steps,
                    "instrumented_ms_per_step": round(inst_ms, 3)}

    if is_batch(name) and not args.no_plain:
        # the plain single-instance path over the same inputs: one wg_tc / wg_sg per instance
        plain_tuples = 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(b.num):
            lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
            if hi > lo:
                _, _, sti = eng.solve(query, src[lo:hi], dst[lo:hi], None)
                plain_tuples += sti["result_tuples"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        extra["single_instance_path"] = {"value": round(plain_tuples / dt, 1), "unit": "tuples/s",
                                         "ms": round(1e3 * dt, 3), "solves": int(b.num)}
        extra["batched_speedup"] = round(value / (plain_tuples / dt), 2)

    out = {
        "metric": "derived tuples/sec per TC/SG fixpoint",
        "value": round(value, 1),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if st["key_bytes"] == 4 else "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(name, name), "name": name,
                   "query": query, "edges": edges, "fixpoint_tuples": st["result_tuples"],
                   "iterations": st["iterations"], "join_candidates": st["join_candidates"],
                   "radix_field_bits": st["field_bits"], "radix_digit_bits": st["digit_bits"],
                   "sort_passes": st["sort_passes"], "host_syncs_per_step": st["host_syncs"]},
        "stage_ms_probe": probe_ms,
        "stage_algorithmic_gb": probe_gb,
        "stage_hbm_frac": probe_frac,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if args.roofline_only:
        out["instrumented"] = True
    out.update(extra)
    eng.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the engine is single-device); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    special = (args.kernel_sweep or args.ablation or args.copy_calibration or args.gather_calibration
               or args.sync_probe)
    default_run = not args.workload_given and not special
    # CPU baselines first: the all-core leg forks worker processes, which must not inherit an
    # initialised GPU runtime (nothing below has touched the GPU yet)
    cpu = {}
    if not args.no_cpu_baseline and not special and args.workload != "served_mix":
        cpu[args.workload] = cpu_baseline(args.workload)
        if default_run and not args.no_extras:
            cpu[SG_EXTRA] = cpu_baseline(SG_EXTRA)
            cpu[BATCH_EXTRA] = cpu_baseline(BATCH_EXTRA, all_core=True)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    if args.copy_calibration:
        # a plain device-to-device copy of known size: what FETCH_SIZE / WRITE_SIZE read for
        # it calibrates the counters against known bytes
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 10}), flush=True)
        return
    if args.gather_calibration:
        # 4-byte reads at random positions (each value read once): with the streamed index
        # (8 B) and output (4 B) it calibrates the counters for scattered reads
        n = (args.gather_calibration << 20) // 4
        g = torch.Generator(device="cuda").manual_seed(11)
        a = torch.arange(n, dtype=torch.int32, device="cuda")
        idx = torch.randperm(n, generator=g, device="cuda")
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        for _ in range(10):
            torch.index_select(a, 0, idx, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"gather_calibration_values": n, "value_bytes": 4, "index_bytes": 8,
                          "algorithmic_read_bytes": 12 * n, "algorithmic_write_bytes": 4 * n,
                          "gathers": 10}), flush=True)
        return
    if args.sync_probe:
        # the two ways to separate the stages of an iteration (Section V-B): a grid-wide
        # barrier inside one persistent launch, or the boundary between two launches
        from paper_2607_17571_amd import wg
        rows = []
        for blocks in (256, 512, 1024, 2048):
            try:
                bar, bar2, bcg, lau = wg.wg_probe_sync_costs(0, blocks, 2000)
            except wg.WgError as e:
                rows.append({"blocks": blocks, "error": str(e)})
                continue
            rows.append({"blocks": blocks, "barrier_us": round(bar, 3), "barrier_two_level_us": round(bar2, 3),
                         "grid_sync_us": round(bcg, 3), "launch_us": round(lau, 3)})
            _progress(f"sync probe: {blocks} blocks: barrier {bar:.3f} us (two-level {bar2:.3f} us, grid sync "
                      f"{bcg:.3f} us), launch {lau:.3f} us")
        print(json.dumps({"sync_probe": rows, "threads_per_block": 256, "rounds": 2000}), flush=True)
        return
    if args.kernel_sweep:
        run_kernel_sweep(args)
        return
    if args.ablation:
        run_ablation(args)
        return
    if args.workload == "served_mix":
        run_served(args)
        return

    def with_cpu(out, name):
        if name in cpu:
            cb, ref = cpu[name]
            if ref is not None and (ref.src.size != out["config"]["fixpoint_tuples"]
                                    or ref.iterations != out["config"]["iterations"]):
                out["cpu_baseline_mismatch"] = True
            out["cpu_baseline"] = cb
        return out

    out = with_cpu(measure(args, args.workload), args.workload)
    if default_run and not args.no_extras:
        # the batched and SG configurations beside the headline, each with its own roofline
        # and CPU baseline (the served mix is not part of this line)
        sub = argparse.Namespace(**vars(args))
        sub.dominant = None
        sub.roofline_only = False
        extra = {}
        _progress(f"extra: {BATCH_EXTRA}")
        sub.steps, sub.warmup = min(args.steps, 3), 1
        extra["batched"] = with_cpu(measure(sub, BATCH_EXTRA), BATCH_EXTRA)
        _progress(f"extra: {SG_EXTRA}")
        sub.steps, sub.warmup = args.steps, min(args.warmup, 3)
        extra["sg"] = with_cpu(measure(sub, SG_EXTRA), SG_EXTRA)
        _progress("extra: served_mix")
        sub.requests, sub.slots, sub.load, sub.hold_after_us = 120, args.slots, 0.7, 0
        sv = measure_served(sub)
        extra["served"] = {k: sv[k] for k in ("value", "unit", "served", "single_instance_path", "load_sweep",
                                              "golden_checks", "config")}
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
