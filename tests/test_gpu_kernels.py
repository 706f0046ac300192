"""The kernel-level entry points (wg_sort_keys, wg_merge_keys) against the oracle, bit-exact:
32- and 64-bit keys, odd and even pass counts, ragged sizes and the empty and single-key
cases."""

import numpy as np
import pytest

import oracle
from paper_2607_17571_amd import wg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def engine():
    eng = wg.Engine(0)
    yield eng
    eng.close()


def _keys(n, bits, dtype, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, size=n, dtype=np.uint64).astype(dtype)


@pytest.mark.parametrize("n,bits,dtype", [
    (0, 30, np.uint32), (1, 30, np.uint32), (2, 30, np.uint32), (4097, 30, np.uint32),
    (1_000_003, 30, np.uint32), (300_001, 24, np.uint32), (65_537, 32, np.uint32),
    (500_001, 48, np.uint64), (123_457, 38, np.uint64), (70_001, 64, np.uint64),
    # tile (4,096 / 2,048 keys) and grid (1,024 blocks x one tile) boundaries
    (4095, 30, np.uint32), (4096, 30, np.uint32), (4097, 30, np.uint32),
    ((1 << 22) - 1, 30, np.uint32), (1 << 22, 30, np.uint32), ((1 << 22) + 1, 30, np.uint32),
    (2047, 48, np.uint64), (2048, 48, np.uint64), (2049, 48, np.uint64),
])
def test_sort_keys(engine, n, bits, dtype):
    import torch

    print(f"[gpu] sort_keys n={n} bits={bits} {np.dtype(dtype).name}", flush=True)
    h = _keys(n, bits, dtype, seed=n + bits)
    keys = torch.from_numpy(h).cuda()
    tmp = torch.empty_like(keys)
    st = engine.sort_keys(keys, tmp, bits)
    torch.cuda.synchronize()
    assert np.array_equal(keys.cpu().numpy(), oracle.sort_keys(h))
    if n > 1:
        rb = engine.sort_config(np.dtype(dtype).itemsize)["digit_bits"]
        assert st["sort_passes"] == -(-bits // rb)


def test_sort_keys_with_duplicates_and_timing(engine):
    import torch

    h = (np.random.default_rng(5).integers(0, 1000, size=2_000_000)).astype(np.uint32)
    keys = torch.from_numpy(h).cuda()
    tmp = torch.empty_like(keys)
    st = engine.sort_keys(keys, tmp, 10, wg.make_options(flags=wg.WG_STAGE_TIMING))
    assert np.array_equal(keys.cpu().numpy(), oracle.sort_keys(h))
    assert st["stage_ms"]["radix_pass"] > 0 and st["stage_bytes"]["radix_pass"] == 2 * 4 * h.size * st["sort_passes"]


@pytest.mark.parametrize("na,nb,bits,dtype", [
    (0, 0, 30, np.uint32), (0, 5, 30, np.uint32), (7, 0, 30, np.uint32), (1, 1, 30, np.uint32),
    (100_003, 77_777, 30, np.uint32), (1_000_000, 3, 32, np.uint32), (250_001, 250_003, 48, np.uint64),
    # tile (2,048 keys) and grid (2,048 blocks x one tile = 2^22) boundaries, ragged splits
    (2047, 0, 30, np.uint32), (2000, 48, 30, np.uint32), (1, 2048, 30, np.uint32),
    (4095, 1, 30, np.uint32), (3000, 1096, 30, np.uint32), (2, 4095, 30, np.uint32),
    ((1 << 22) - 7, 6, 30, np.uint32), ((1 << 21), 1 << 21, 30, np.uint32),
    ((1 << 22) - 1, 2, 30, np.uint32), (1024, 1023, 48, np.uint64), (1 << 21, (1 << 21) + 1, 48, np.uint64),
])
def test_merge_keys(engine, na, nb, bits, dtype):
    import torch

    print(f"[gpu] merge_keys na={na} nb={nb} {np.dtype(dtype).name}", flush=True)
    a = np.sort(_keys(na, bits, dtype, seed=na + 1))
    b = np.sort(_keys(nb, bits, dtype, seed=nb + 2))
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    out = torch.empty(max(1, na + nb), dtype=ta.dtype, device="cuda")
    engine.merge_keys(ta, tb, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy()[: na + nb], oracle.merge_runs(a, b))


def test_kernel_calls_reject_bad_arguments(engine):
    import torch

    k = torch.zeros(10, dtype=torch.uint32, device="cuda")
    for bits in (0, 33):
        with pytest.raises(wg.WgError) as ei:
            engine.sort_keys(k, torch.empty_like(k), bits)
        assert ei.value.status == wg.WG_ERR_INVALID_ARG


def test_kernel_calls_leave_the_result_valid(engine):
    import torch
    from paper_2607_17571_amd import inputs

    src, dst = inputs.erdos_renyi(500, 700, seed=3)
    s, d, st = engine.tc(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    ref = oracle.tc(src, dst)
    k = torch.from_numpy(_keys(100_000, 30, np.uint32, 9)).cuda()
    engine.sort_keys(k, torch.empty_like(k), 30)
    assert np.array_equal(s.cpu().numpy(), ref.src) and np.array_equal(d.cpu().numpy(), ref.dst)


def test_sync_probe():
    """The synchronisation probe (grid-wide barrier in one cooperative launch against a
    dependent launch) returns positive costs and rejects bad arguments."""
    print("[gpu] sync probe 256 blocks", flush=True)
    bar, bar2, bcg, lau = wg.wg_probe_sync_costs(0, 256, 200)
    assert 0 < bar < 1000 and 0 < bar2 < 1000 and 0 < bcg < 1000 and 0 < lau < 1000
    # one block: every barrier is a single arrival
    bar, bar2, bcg, lau = wg.wg_probe_sync_costs(0, 1, 50)
    assert bar < 1000 and bar2 < 1000 and bcg < 1000 and 0 < lau < 1000
    for blocks, rounds in ((0, 10), (4096, 10), (256, 0)):
        with pytest.raises(wg.WgError) as ei:
            wg.wg_probe_sync_costs(0, blocks, rounds)
        assert ei.value.status == wg.WG_ERR_INVALID_ARG
