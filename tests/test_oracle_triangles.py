"""Pins of the triangle-counting oracle against definitions independent of its join.

* trace(A^3) of the dense 0/1 adjacency matrix (closed walks of length 3 = bindings
  (a, b, c) of the rule), on random graphs, with and without self-loops and duplicates;
* trace of a sparse matrix product (scipy) on a larger R-MAT graph;
* closed forms: a directed 3-cycle, longer cycles, complete directed graphs, a single
  self-loop, a two-cycle, an empty graph;
* a planted mistake (dropping the closing-edge direction) must fail a pin.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_2607_17571_amd import inputs


def dense_trace_a3(src, dst, n):
    A = np.zeros((n, n), dtype=np.int64)
    A[np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64)] = 1
    return int(np.trace(A @ A @ A))


@settings(max_examples=120, deadline=None)
@given(n=st.integers(1, 30), m=st.integers(0, 150), seed=st.integers(0, 10**6))
def test_equals_trace_of_a_cubed(n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.uint32)  # self-loops and duplicates allowed
    dst = rng.integers(0, n, m).astype(np.uint32)
    count, _ = oracle.triangles(src, dst)
    assert count == dense_trace_a3(src, dst, n)


def test_sparse_trace_on_rmat():
    src, dst = inputs.rmat(11, 4000, *inputs.RMAT_ABCD, seed=12)
    n = 1 << 11
    A = sp.csr_matrix((np.ones(src.size, dtype=np.int64), (src.astype(np.int64), dst.astype(np.int64))),
                      shape=(n, n))
    A.data[:] = 1  # duplicates collapse
    count, _ = oracle.triangles(src, dst)
    assert count == int((A @ A @ A).diagonal().sum())


@pytest.mark.parametrize("k", [3, 4, 5, 9])
def test_directed_cycles(k):
    src, dst = inputs.cycle(k)
    count, two = oracle.triangles(src, dst)
    assert count == (3 if k == 3 else 0)
    assert two == k


@pytest.mark.parametrize("k", [2, 3, 4, 7])
def test_complete_directed_graph(k):
    a, b = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    keep = a != b
    count, _ = oracle.triangles(a[keep].astype(np.uint32), b[keep].astype(np.uint32))
    assert count == k * (k - 1) * (k - 2)


def test_small_cases():
    assert oracle.triangles([5], [5]) == (1, 1)          # (5,5,5)
    assert oracle.triangles([0, 1], [1, 0])[0] == 0      # a two-cycle closes no triangle
    assert oracle.triangles([], []) == (0, 0)
    assert oracle.triangles([0, 0, 1, 2], [1, 1, 2, 0])[0] == 3  # duplicates collapse


def test_planted_mistake_fails_a_pin():
    """Closing with (a, c) instead of (c, a) counts transitive triangles, not cycles."""
    def wrong(src, dst):
        E = np.unique((np.asarray(src, np.uint64) << np.uint64(32)) | np.asarray(dst, np.uint64))
        s, d = E >> np.uint64(32), E & np.uint64(0xFFFFFFFF)
        total = 0
        for a, b in zip(s, d):
            for c in d[s == b]:
                total += int(((a << np.uint64(32)) | c) in set(E.tolist()))
        return total
    src, dst = inputs.rmat(6, 150, *inputs.RMAT_ABCD, seed=3)
    assert wrong(src, dst) != dense_trace_a3(src, dst, 64)
    assert oracle.triangles(src, dst)[0] == dense_trace_a3(src, dst, 64)
