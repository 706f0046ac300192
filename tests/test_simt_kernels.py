"""Kernel text on the CPU SIMT shim (tests/simt): concurrency and bounds checks that a
GPU run cannot give.

Regression test: the early exit of a launch is decided once per block.

Block 0 of the row pass's gather records the iteration and, for an empty delta, sets the
fixpoint flag that every block tests at its start; the join's emit and the compaction's
gather likewise report overflows.  When the threads of one block tested such a flag at
different moments, part of the block returned and the rest went on into block-wide scans
whose partial sums the others never wrote (on the GPU: garbage prefix sums, then stores at
garbage positions).  This runs the current kernel text of the row pass and its gather on
the CPU SIMT shim under tests/simt (every GPU thread a fiber, blocks concurrently on OS
threads with their own LDS, AddressSanitizer on), with the fixpoint reached and with a
non-empty delta, many times: every run must give the plain set difference and no block
may split.
"""

import os
import platform
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIMT = os.path.join(ROOT, "tests", "simt")
CSRC = os.path.join(ROOT, "paper_2607_17571_amd", "csrc")
KERNELS = ["const:kRowWordsMax", "const:kRowItems", "const:kRowTile", "nth_set_bit", "or_sorted_runs", "const:kRowFan",
           "row_search", "k_row_diff",
           "record_iteration", "k_row_gather"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or platform.machine() != "x86_64",
                                reason="needs g++ on x86-64 (the shim switches fibers in x86-64 assembly)")


def _build(d, harness_src, inc_name, names):
    inc = subprocess.run([sys.executable, os.path.join(SIMT, "extract.py"), os.path.join(CSRC, "wg_kernels.hip"),
                          *names], capture_output=True, text=True, check=True).stdout
    (d / inc_name).write_text(inc)
    exe = d / os.path.splitext(harness_src)[0]
    subprocess.run(["g++", "-std=c++20", "-O1", "-g", "-DSIMT_STACK=131072", "-fsanitize=address",
                    "-fno-omit-frame-pointer",
                    f"-I{d}", f"-I{SIMT}", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}", "-pthread",
                    os.path.join(SIMT, harness_src), "-o", str(exe)], check=True, capture_output=True)
    return exe


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("simt"), "row_harness.cpp", "row.inc", KERNELS)


def _write(path, cand, a, b, w):
    with open(path, "wb") as f:
        np.array([cand.size, a.size, b.size, w, 4], dtype=np.uint64).tofile(f)
        cand.astype(np.uint32).tofile(f)
        a.astype(np.uint32).tofile(f)
        b.astype(np.uint32).tofile(f)


def _case(seed, empty_delta):
    rng = np.random.default_rng(seed)
    w = 8
    rows = np.sort(rng.choice(1 << 12, size=300, replace=False)).astype(np.uint64)
    full = np.unique(np.concatenate([(r << np.uint64(w)) | rng.integers(0, 1 << w, size=int(rng.integers(1, 60)),
                                                                       dtype=np.uint64) for r in rows]))
    cand = []
    for r in rows:
        mine = full[(full >> np.uint64(w)) == r]
        if empty_delta:
            d = rng.choice(mine, size=int(rng.integers(1, 40)))  # every candidate already in Full
        else:
            d = (r << np.uint64(w)) | rng.integers(0, 1 << w, size=int(rng.integers(1, 40)), dtype=np.uint64)
        cand.append(d)
    cand = np.concatenate(cand)
    nb = full.size // 5
    perm = rng.permutation(full.size)
    return cand, np.sort(full[perm[nb:]]), np.sort(full[perm[:nb]]), w


@pytest.mark.parametrize("empty_delta", [True, False], ids=["fixpoint", "delta"])
def test_row_gather_blocks_never_split(harness, tmp_path, empty_delta):
    cand, a, b, w = _case(7 if empty_delta else 8, empty_delta)
    path = tmp_path / "in.bin"
    _write(path, cand, a, b, w)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(harness), str(path), "64", "8", "20"], capture_output=True, text=True, env=env,
                       timeout=300)
    assert "simt:" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert r.stdout.count("ok ") == 20


COMPACT = ["drop_present", "drop_present_sampled", "compact_span", "k_compact_local", "record_iteration", "compact_gather",
           "k_compact_gather"]


@pytest.fixture(scope="module")
def compact_harness(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("simt_c"), "compact_harness.cpp", "compact.inc", COMPACT)


def _compact_case(seed, key_bytes, per_item):
    """Sorted candidates (half of them keys of Full, with duplicates) against Full split into
    runs A and B; about `per_item` keys of Full per candidate, so that the tiles' windows are
    staged whole (< 1) or searched through staged samples (more)."""
    rng = np.random.default_rng(seed)
    bits = 30 if key_bytes == 4 else 48
    full = np.unique(rng.integers(0, 1 << bits, size=300_000, dtype=np.uint64))
    nc = max(2, int(full.size / per_item))
    new = rng.integers(0, 1 << bits, size=nc - nc // 2, dtype=np.uint64)
    cand = np.sort(np.concatenate([rng.choice(full, size=nc // 2), new, rng.choice(new, size=nc // 8)]))
    rng.shuffle(full)
    nb = full.size // 4
    return cand, np.sort(full[nb:]), np.sort(full[:nb])


@pytest.mark.parametrize("key_bytes,per_item,items", [(4, 0.5, 8), (4, 6, 8), (8, 6, 4), (8, 300, 8)],
                         ids=["u32-staged", "u32-sampled", "u64-sampled-narrow", "u64-sampled-sparse"])
def test_compaction_windows(compact_harness, tmp_path, key_bytes, per_item, items):
    cand, a, b = _compact_case(11 + items, key_bytes, per_item)
    path = tmp_path / "in.bin"
    dt = np.uint32 if key_bytes == 4 else np.uint64
    with open(path, "wb") as f:
        np.array([cand.size, a.size, b.size, 15 if key_bytes == 4 else 24, key_bytes], dtype=np.uint64).tofile(f)
        cand.astype(dt).tofile(f)
        a.astype(dt).tofile(f)
        b.astype(dt).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(compact_harness), str(path), "64", "8", "3", str(items)], capture_output=True, text=True,
                       env=env, timeout=300)
    assert "simt:" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert r.stdout.count("ok ") == 3


SEG = ["const:kSmallSortThreads", "shfl_xor_key", "bitonic_keep", "xor_lanes32", "xor_lanes", "wave_stage", "block_bitonic_sort", "const:kSegTile",
       "const:kSegBitonicMax", "const:kSegLongBytes", "k_seg_sort"]


@pytest.fixture(scope="module")
def seg_harness(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("simt_s"), "seg_harness.cpp", "seg.inc", SEG)


@pytest.mark.parametrize("key_bytes,lens", [(4, (1, 6)), (4, (1, 400)), (8, (1, 2000))],
                         ids=["u32-short-rows", "u32-rows-to-400", "u64-rows-to-2000"])
def test_segmented_sort(seg_harness, tmp_path, key_bytes, lens):
    """The segmented sort of row-grouped candidates (rows ascending, each row's keys in any
    order), 1,024 threads a block, blocks concurrent: the output is the keys sorted.  (A tile
    plus the tail of its last row stays within the one-block network here; longer rows are
    the long-row pass's.)"""
    rng = np.random.default_rng(31 + lens[1])
    w = 15 if key_bytes == 4 else 24
    rows = np.sort(rng.choice(1 << 16, size=400, replace=False)).astype(np.uint64)
    keys = np.concatenate([(r << np.uint64(w)) | rng.integers(0, 1 << w, size=int(rng.integers(*lens)),
                                                              dtype=np.uint64) for r in rows])
    path = tmp_path / "in.bin"
    with open(path, "wb") as f:
        np.array([keys.size, w, key_bytes], dtype=np.uint64).tofile(f)
        keys.astype(np.uint32 if key_bytes == 4 else np.uint64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(seg_harness), str(path), "64", "8", "2"], capture_output=True, text=True, env=env,
                       timeout=300)
    assert "simt:" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert r.stdout.count("ok ") == 2


# ---------------------------------------------------------------------------
# The tail loop (one block looping over whole iterations) and the fold after it.
# ---------------------------------------------------------------------------
TAIL = ["const:kNoRow", "const:kSmallSortThreads", "shfl_xor_key", "bitonic_keep", "xor_lanes32", "xor_lanes", "wave_stage", "block_bitonic_sort", "struct:OneBlockJoin",
        "lds_bounds", "lds_lower_bounds", "lds_upper_bounds",
        "one_block_count", "one_block_emit", "const:kTailFenceBytes", "drop_found", "k_tail_loop",
        "wave_merge_path", "merge_tiles_to", "merge_tiles", "k_tail_fold"]


@pytest.fixture(scope="module")
def tail_harness(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("simt_tail"), "tail_harness.cpp", "tail.inc", TAIL)


def _tail_case(tail_harness, tmp_path, query, src, dst, kb, split, jstep, grid=7):
    """Runs the tail loop from the seed to the fixpoint (the seed's Full split at random into
    runs A and B) and compares every iteration's delta size, the candidate total and the
    result with the oracle."""
    import oracle
    from oracle import seminaive as sn

    w = max(1, int(max(src.max(), dst.max())).bit_length())
    assert 2 * w <= 8 * kb
    E = sn.sort_unique(sn.pack(src, dst))
    seed = E if query == 0 else sn.sort_unique(sn.sg_base(*sn.edge_index(E)))
    ref = oracle.tc(src, dst) if query == 0 else oracle.sg(src, dst)

    def rekey(k):  # the oracle's 32-bit fields -> w-bit fields
        return ((k >> np.uint64(32)) << np.uint64(w)) | (k & np.uint64(0xFFFFFFFF))
    E, seed = rekey(E), rekey(seed)
    rng = np.random.default_rng(len(seed))
    pick = rng.random(seed.size) < split
    A, B = np.sort(seed[~pick]), np.sort(seed[pick])
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([query, w, kb, E.size, A.size, B.size], dtype=np.uint64).tofile(f)
        for a in (E, A, B):
            a.astype(np.uint64).tofile(f)
    r = subprocess.run([str(tail_harness), str(inp), str(out), str(grid), "8", str(jstep)], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    got = np.fromfile(out, dtype=np.uint64)
    iters = int(got[0])
    NC = got[1:1 + 2 * iters].reshape(iters, 2)
    nf = int(got[1 + 2 * iters])
    full = got[2 + 2 * iters:2 + 2 * iters + nf]
    launches, at_records, at_run = (int(x) for x in got[2 + 2 * iters + nf:])
    assert iters == ref.iterations
    assert [int(x) for x in NC[:, 0]] == list(ref.delta_sizes[1:])
    assert int(NC[:, 1].sum()) == ref.candidates
    want = (ref.src.astype(np.uint64) << np.uint64(w)) | ref.dst.astype(np.uint64)
    np.testing.assert_array_equal(full, np.sort(want))
    return launches, at_records, at_run


@pytest.mark.parametrize("kb", [4, 8])
def test_tail_loop_tc_to_the_fixpoint(tail_harness, tmp_path, kb):
    from paper_2607_17571_amd import inputs
    src, dst = inputs.erdos_renyi(60, 75, seed=3)
    launches, at_records, _ = _tail_case(tail_harness, tmp_path, 0, src, dst, kb, split=0.3, jstep=3)
    assert launches > 1 and at_records > 0  # the record bound stopped it and it went on


def test_tail_loop_tc_fills_its_run(tail_harness, tmp_path):
    """A closure beyond run T's capacity: T fills, the fold merges it into B, the next
    launch starts from there."""
    from paper_2607_17571_amd import inputs
    src, dst = inputs.chain(150)  # 11,175 tuples, a few hundred new per iteration
    launches, _, at_run = _tail_case(tail_harness, tmp_path, 0, src, dst, 4, split=0.0, jstep=400)
    assert at_run > 0


@pytest.mark.parametrize("kb,n,m", [(4, 4000, 3000), (8, 2400, 1800)])
def test_tail_loop_tc_run_a_beyond_its_fences(tail_harness, tmp_path, kb, n, m):
    """About 90% of the seed in run A: more keys than its LDS fences hold (2,048 32-bit or
    1,024 64-bit samples), so every search of A takes the fences and then bisects a stretch
    in HBM; the seed delta and every iteration still fit one block."""
    from paper_2607_17571_amd import inputs
    src, dst = inputs.erdos_renyi(n, m, seed=8)
    assert 0.9 * np.unique((src.astype(np.uint64) << np.uint64(32)) | dst).size > (8192 // kb)
    _tail_case(tail_harness, tmp_path, 0, src, dst, kb, split=0.1, jstep=40)


def test_tail_loop_sg(tail_harness, tmp_path):
    from paper_2607_17571_amd import inputs
    src, dst = inputs.erdos_renyi(40, 60, seed=5)
    _tail_case(tail_harness, tmp_path, 1, src, dst, 4, split=0.5, jstep=2)
