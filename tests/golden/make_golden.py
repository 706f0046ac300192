"""Write expected fixpoint summaries for the full-size workloads.

Every value stored here comes from the CPU oracle (``oracle/``) run on the seeded
inputs of ``paper_2607_17571_amd.inputs``; nothing is taken from the GPU path.
Run from the repository root:

    python tests/golden/make_golden.py [workload ...]

Output: tests/golden/fixpoints.json, one record per workload with the fixpoint
size, the iteration count, |Delta^i| per iteration, the candidate total and the
sha256 of the result bytes (little-endian uint32 src array followed by the dst
array, lexicographically sorted).  Batched workloads (names with "_batch_") store the
total size, the largest instance's iteration count, the sha256 of the per-instance
results concatenated in instance order (local ids; src bytes then dst bytes) and the
sha256 of the result offsets (num + 1 little-endian int64).  The served mix
("served_mix_<requests>_seed<seed>") stores one record per request: query, edges, the
fixpoint size, the iteration count and the sha256 of its result bytes.
"""

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2607_17571_amd import inputs  # noqa: E402

DEFAULT = ["tc_er_2000", "sg_er_500k", "tc_rmat_s15", "tc_rmat_s16", "tc_rmat_s15_ids24", "tc_grid_100",
           "tc_batch_er_256", "sg_batch_er_256", "tc_batch_er_4096", "served_mix_120_seed5"]


def summarise_batch(results):
    import numpy as np

    src = np.concatenate([r.src for r in results]).astype("<u4")
    dst = np.concatenate([r.dst for r in results]).astype("<u4")
    offsets = np.zeros(len(results) + 1, dtype="<i8")
    offsets[1:] = np.cumsum([r.src.size for r in results])
    return {"size": int(src.size), "iterations": max(r.iterations for r in results),
            "sha256": hashlib.sha256(src.tobytes() + dst.tobytes()).hexdigest(),
            "offsets_sha256": hashlib.sha256(offsets.tobytes()).hexdigest(),
            "instances": len(results)}


def summarise(r):
    h = hashlib.sha256(r.src.astype("<u4").tobytes() + r.dst.astype("<u4").tobytes()).hexdigest()
    return {"size": int(r.src.size), "iterations": r.iterations,
            "delta_sizes": r.delta_sizes, "candidates": r.candidates, "sha256": h}


def served_mix(name):
    """Per-request records of the served mix ``served_mix_<requests>_seed<seed>``."""
    _, _, num, seed = name.split("_")
    reqs = inputs.served_requests(int(num), seed=int(seed[len("seed"):]))
    recs = []
    for i, r in enumerate(reqs):
        t0 = time.time()
        f = oracle.tc(r.src, r.dst) if r.query == "tc" else oracle.sg(r.src, r.dst)
        rec = summarise(f)
        del rec["delta_sizes"]
        rec.update(query=r.query, kind=r.kind, n=int(r.n), edges=int(r.src.size))
        recs.append(rec)
        print(f"{name}[{i}] {r.query} {r.kind} n={r.n}: |fixpoint|={rec['size']} "
              f"({time.time() - t0:.1f} s)", flush=True)
    return {"requests": recs}


def main(names):
    path = os.path.join(HERE, "fixpoints.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        if name.startswith("served_mix_"):
            data[name] = served_mix(name)
            with open(path, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
                f.write("\n")
            continue
        if "_batch_" in name:
            t0 = time.time()
            query, b = inputs.batch_workload(name)
            fn = oracle.tc_batch if query == "tc" else oracle.sg_batch
            rec = summarise_batch(fn(b.src, b.dst, b.offsets))
            rec["query"] = query
            rec["edges"] = int(b.src.size)
            data[name] = rec
            print(f"{name}: |fixpoint|={rec['size']} iterations={rec['iterations']} "
                  f"({time.time() - t0:.1f} s)", flush=True)
            with open(path, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
                f.write("\n")
            continue
        w = inputs.workload(name)
        t0 = time.time()
        r = oracle.tc(w.src, w.dst) if w.query == "tc" else oracle.sg(w.src, w.dst)
        rec = summarise(r)
        rec["query"] = w.query
        rec["edges"] = int(w.src.size)
        data[name] = rec
        if w.query == "sg":
            data[name + "_irreflexive"] = dict(
                summarise(oracle.sg(w.src, w.dst, irreflexive=True)), query="sg", edges=int(w.src.size))
        print(f"{name}: |fixpoint|={rec['size']} iterations={rec['iterations']} "
              f"({time.time() - t0:.1f} s)", flush=True)
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or DEFAULT)
