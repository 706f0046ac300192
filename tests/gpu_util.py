"""Helpers shared by the GPU parity tests (host-side marshalling only)."""

import hashlib
import sys

import numpy as np


def to_gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32)).to("cuda")


def run(engine, query, src, dst, options=None):
    """Solve on the GPU through the C ABI; returns (src, dst, stats) with numpy outputs."""
    print(f"[gpu] {query} m={len(src)}", flush=True, file=sys.stderr)
    s, d, st = engine.solve(query, to_gpu(src), to_gpu(dst), options)
    return s.cpu().numpy(), d.cpu().numpy(), st


def digest(src, dst):
    return hashlib.sha256(np.asarray(src, dtype="<u4").tobytes() + np.asarray(dst, dtype="<u4").tobytes()).hexdigest()


def assert_same(gpu_src, gpu_dst, gpu_stats, ref):
    """Element-by-element equality with the oracle, plus iteration count and delta sizes."""
    assert gpu_src.shape == ref.src.shape, (gpu_src.shape, ref.src.shape)
    np.testing.assert_array_equal(gpu_src, ref.src)
    np.testing.assert_array_equal(gpu_dst, ref.dst)
    assert gpu_stats["iterations"] == ref.iterations
    assert gpu_stats["delta_sizes"] == ref.delta_sizes
    assert gpu_stats["join_candidates"] == ref.candidates
