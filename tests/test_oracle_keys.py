"""Pins of the single-stage oracle (sort and merge of key arrays) against independent
definitions: Python's own sorted() and heapq.merge, hand examples, and invariants."""

import heapq

import numpy as np

import oracle


def test_sort_keys_hand_example():
    k = np.array([5, 3, 3, 0xFFFFFFFF, 0, 7], dtype=np.uint32)
    assert oracle.sort_keys(k).tolist() == [0, 3, 3, 5, 7, 0xFFFFFFFF]


def test_sort_keys_matches_python_sorted():
    rng = np.random.default_rng(31)
    for n in (0, 1, 2, 17, 1000):
        for dt, hi in ((np.uint32, 1 << 32), (np.uint64, 1 << 48)):
            k = rng.integers(0, hi, size=n, dtype=np.uint64).astype(dt)
            out = oracle.sort_keys(k)
            assert out.dtype == dt
            assert out.tolist() == sorted(k.tolist())


def test_sort_keys_keeps_the_multiset_and_orders_it():
    rng = np.random.default_rng(32)
    k = rng.integers(0, 50, size=5000).astype(np.uint32)  # many duplicates
    out = oracle.sort_keys(k)
    assert np.all(out[:-1] <= out[1:])
    v1, c1 = np.unique(k, return_counts=True)
    v2, c2 = np.unique(out, return_counts=True)
    assert np.array_equal(v1, v2) and np.array_equal(c1, c2)


def test_merge_runs_hand_examples():
    a = np.array([1, 4, 9], dtype=np.uint32)
    b = np.array([2, 3, 10, 11], dtype=np.uint32)
    assert oracle.merge_runs(a, b).tolist() == [1, 2, 3, 4, 9, 10, 11]
    assert oracle.merge_runs(a, b[:0]).tolist() == [1, 4, 9]
    assert oracle.merge_runs(a[:0], b).tolist() == [2, 3, 10, 11]
    assert oracle.merge_runs(np.array([5], np.uint32), np.array([5], np.uint32)).tolist() == [5, 5]


def test_merge_runs_matches_heapq_merge():
    rng = np.random.default_rng(33)
    for na, nb in ((0, 0), (1, 0), (0, 3), (7, 5), (300, 1000)):
        a = np.sort(rng.integers(0, 1 << 40, size=na, dtype=np.uint64))
        b = np.sort(rng.integers(0, 1 << 40, size=nb, dtype=np.uint64))
        assert oracle.merge_runs(a, b).tolist() == list(heapq.merge(a.tolist(), b.tolist()))
