"""The engine's allocator hook (wg_engine_create_ex): every device buffer comes from the
caller's allocator -- here torch's caching allocator -- and results stay bit-exact."""

import sys

import numpy as np
import pytest

import oracle
from paper_2607_17571_amd import inputs, wg
from tests.gpu_util import assert_same, to_gpu

pytestmark = pytest.mark.gpu


def _solve(eng, query, src, dst, opts=None):
    print(f"[gpu] hooked {query} m={len(src)}", flush=True, file=sys.stderr)
    s, d, st = eng.solve(query, to_gpu(src), to_gpu(dst), opts)
    return s.cpu().numpy(), d.cpu().numpy(), st


def test_torch_allocator_supplies_every_buffer():
    import torch

    hook = wg.TorchAllocator(0)
    eng = wg.Engine(0, allocator=hook)
    try:
        fixed = hook.allocs
        assert fixed >= 6 and hook.frees == 0  # control block, block totals, radix counts, hits
        src, dst = inputs.rmat(11, 1800, *inputs.RMAT_ABCD, seed=41)
        s, d, st = _solve(eng, "tc", src, dst)
        assert_same(s, d, st, oracle.tc(src, dst))
        after_small = hook.allocs
        assert after_small > fixed  # relation buffers, records, index
        # a larger input grows the buffers mid-solve: more calls, stream-ordered frees
        w = inputs.workload("tc_rmat_s15")
        big_s, big_d, big_st = _solve(eng, "tc", w.src, w.dst)
        assert hook.allocs > after_small and hook.frees > 0
        assert big_st["result_tuples"] == 49858560
        # the memory torch handed out is what the engine holds
        held = sum(b for b, _ in hook.live.values())
        assert held >= 8 * big_st["result_tuples"] // 2
        s, d, st = _solve(eng, "sg", src, dst)
        assert_same(s, d, st, oracle.sg(src, dst))
    finally:
        eng.close()
    assert hook.frees == hook.allocs and not hook.live


class _LimitedAllocator(wg.TorchAllocator):
    """Refuses every allocation after the first `limit` (counts the refusals)."""

    def __init__(self, limit):
        super().__init__(0)
        self.limit = limit

    def _on_alloc(self, nbytes, stream, user):
        if self.allocs >= self.limit:
            self.failed += 1
            return None
        return super()._on_alloc(nbytes, stream, user)


def test_allocator_failure_is_out_of_memory_and_engine_stays_usable():
    src, dst = inputs.erdos_renyi(3000, 2800, seed=42)
    hook = _LimitedAllocator(limit=8)
    eng = wg.Engine(0, allocator=hook)
    try:
        with pytest.raises(wg.WgError) as ei:
            _solve(eng, "tc", src, dst)
        assert ei.value.status == wg.WG_ERR_OUT_OF_MEMORY and hook.failed >= 1
        hook.limit = 1 << 30
        s, d, st = _solve(eng, "tc", src, dst)
        assert_same(s, d, st, oracle.tc(src, dst))
    finally:
        eng.close()
    assert hook.frees == hook.allocs


def test_default_allocator_is_stream_ordered_and_exact():
    """NULL allocator: hipMallocAsync / hipFreeAsync on the solve's stream; growth from small
    buffers and a side stream keep the results exact."""
    import torch

    eng = wg.Engine(0)
    try:
        side = torch.cuda.Stream()
        w = inputs.workload("tc_rmat_s15")
        ref = oracle.tc(*inputs.rmat(10, 900, *inputs.RMAT_ABCD, seed=43))
        with torch.cuda.stream(side):
            s, d, st = eng.solve("tc", to_gpu(ref.src), to_gpu(ref.dst))  # closure of a closure
            big = eng.solve("tc", to_gpu(w.src), to_gpu(w.dst))[2]
        side.synchronize()
        assert big["result_tuples"] == 49858560
        ref2 = oracle.tc(ref.src, ref.dst)
        np.testing.assert_array_equal(s.cpu().numpy(), ref2.src)
        np.testing.assert_array_equal(d.cpu().numpy(), ref2.dst)
    finally:
        eng.close()
