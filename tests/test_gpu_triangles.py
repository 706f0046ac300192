"""Triangle counting (wg_triangles) against the oracle, through the C ABI.

The count of bindings of triangle(a,b,c) <- edge(a,b), edge(b,c), edge(c,a) is an exact
integer: the bar is equality with the oracle (itself pinned to trace(A^3)), and the
number of two-paths the join expanded must equal the oracle's.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2607_17571_amd import inputs
from paper_2607_17571_amd import wg
from tests.gpu_util import assert_same, run, to_gpu

pytestmark = pytest.mark.gpu


def gpu_triangles(engine, src, dst, options=None):
    print(f"[gpu] triangles m={len(src)}", flush=True, file=sys.stderr)
    return engine.triangles(to_gpu(src), to_gpu(dst), options)


@pytest.mark.parametrize("make", [
    lambda: inputs.cycle(3), lambda: inputs.cycle(7), lambda: inputs.complete_dag(30),
    lambda: (np.array([4], np.uint32), np.array([4], np.uint32)),
    lambda: (np.array([0, 1, 1, 2, 2], np.uint32), np.array([1, 2, 2, 0, 0], np.uint32)),
])
def test_small_shapes(engine, make):
    src, dst = make()
    count, st = gpu_triangles(engine, src, dst)
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_er(engine, seed):
    src, dst = inputs.erdos_renyi(3000, 9000, seed=seed)
    count, st = gpu_triangles(engine, src, dst)
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two


@pytest.mark.parametrize("scale,m", [(10, 4000), (13, 40000), (15, 200000)])
def test_rmat_hubs(engine, scale, m):
    """Hub-heavy graphs: many two-paths per hub edge, spread over the emit tiles."""
    src, dst = inputs.rmat(scale, m, *inputs.RMAT_ABCD, seed=scale)
    count, st = gpu_triangles(engine, src, dst)
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two


def test_wide_ids_and_self_loops(engine):
    src, dst = inputs.scatter_ids(*inputs.rmat(11, 9000, *inputs.RMAT_ABCD, seed=8), 30, seed=2)
    src = np.concatenate([src, src[:50]])  # self-loops on 50 vertices and duplicates
    dst = np.concatenate([dst, src[:50]])
    count, st = gpu_triangles(engine, src, dst)
    ref, two = oracle.triangles(src, dst)
    assert st["key_bytes"] == 8
    assert count == ref and st["join_candidates"] == two


def test_empty_and_repeat(engine):
    count, _ = gpu_triangles(engine, np.empty(0, np.uint32), np.empty(0, np.uint32))
    assert count == 0
    src, dst = inputs.cycle(3)
    assert gpu_triangles(engine, src, dst)[0] == 3
    assert gpu_triangles(engine, src, dst)[0] == 3


@pytest.mark.parametrize("scale,m", [(10, 4000), (13, 40000)])
def test_hash_join_variant(engine, scale, m):
    src, dst = inputs.rmat(scale, m, *inputs.RMAT_ABCD, seed=scale)
    count, st = gpu_triangles(engine, src, dst, wg.make_options(flags=wg.WG_JOIN_HASH))
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two


@pytest.mark.parametrize("scale,m", [(10, 4000), (13, 40000)])
def test_fair_hash_join_variant(engine, scale, m):
    """Hashed row lookups and a pair set for the closing edges: the same counts."""
    src, dst = inputs.rmat(scale, m, *inputs.RMAT_ABCD, seed=scale)
    count, st = gpu_triangles(engine, src, dst, wg.make_options(flags=wg.WG_JOIN_HASH_ROWS))
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two


def test_fair_hash_join_self_loops_and_wide_ids(engine):
    src, dst = inputs.scatter_ids(*inputs.rmat(10, 3000, *inputs.RMAT_ABCD, seed=3), 30, seed=6)
    src = np.concatenate([src, src[:50]])
    dst = np.concatenate([dst, src[:50]])  # self-loops
    count, st = gpu_triangles(engine, src, dst, wg.make_options(flags=wg.WG_JOIN_HASH_ROWS))
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two


def test_variant_does_not_leak_into_the_next_solve(engine):
    """A solve without a join flag after one with the fair hash (and the other way round)
    probes the index it built itself, not the previous solve's table."""
    src, dst = inputs.rmat(10, 4000, *inputs.RMAT_ABCD, seed=11)
    ref, two = oracle.triangles(src, dst)
    for flags in (wg.WG_JOIN_HASH_ROWS, wg.WG_SPARSE_INDEX, wg.WG_JOIN_HASH_ROWS, 0, wg.WG_JOIN_HASH,
                  wg.WG_JOIN_HASH_ROWS, 0):
        count, st = gpu_triangles(engine, src, dst, wg.make_options(flags=flags))
        assert (count, st["join_candidates"]) == (ref, two), flags
    a, b = inputs.rmat(11, 1800, *inputs.RMAT_ABCD, seed=9)
    want = oracle.tc(a, b)
    for flags in (wg.WG_JOIN_HASH_ROWS, 0, wg.WG_JOIN_HASH_ROWS | wg.WG_ITER_GRAPH, wg.WG_ITER_GRAPH):
        s, d, st = run(engine, "tc", a, b, wg.make_options(flags=flags))
        assert_same(s, d, st, want)


@pytest.mark.parametrize("scale,m", [(10, 4000), (12, 20000)])
def test_sparse_index_variant(engine, scale, m):
    src, dst = inputs.rmat(scale, m, *inputs.RMAT_ABCD, seed=scale + 1)
    count, st = gpu_triangles(engine, src, dst, wg.make_options(flags=wg.WG_SPARSE_INDEX))
    ref, two = oracle.triangles(src, dst)
    assert count == ref and st["join_candidates"] == two
