"""Seeded input generators: determinism, exact sizes, no loops or duplicates, R-MAT skew."""

import hashlib

import numpy as np
import pytest

from paper_2607_17571_amd import inputs


def digest(src, dst):
    return hashlib.sha256(src.tobytes() + dst.tobytes()).hexdigest()


@pytest.mark.parametrize("gen", [
    lambda: inputs.erdos_renyi(2000, 1900, seed=1),
    lambda: inputs.rmat(12, 3000, *inputs.RMAT_ABCD, seed=2),
])
def test_same_seed_same_bytes(gen):
    a, b = gen(), gen()
    assert digest(*a) == digest(*b)


def test_different_seed_different_bytes():
    assert digest(*inputs.erdos_renyi(500, 400, seed=1)) != digest(*inputs.erdos_renyi(500, 400, seed=2))


@pytest.mark.parametrize("n,m", [(2, 2), (10, 90), (2000, 1900), (500_000, 450_000)])
def test_er_exact_m_no_loops_no_duplicates(n, m):
    s, d = inputs.erdos_renyi(n, m, seed=3)
    assert s.dtype == np.uint32 and d.dtype == np.uint32
    assert s.size == m and d.size == m
    assert np.all(s != d)
    assert np.unique((s.astype(np.uint64) << np.uint64(32)) | d).size == m
    assert s.max(initial=0) < n and d.max(initial=0) < n


def test_er_rejects_impossible_m():
    with pytest.raises(ValueError):
        inputs.erdos_renyi(3, 7, seed=0)


def test_rmat_exact_m_and_quadrant_skew():
    scale, m = 12, 20000
    s, d = inputs.rmat(scale, m, *inputs.RMAT_ABCD, seed=4)
    assert s.size == m and np.all(s != d)
    assert np.unique((s.astype(np.uint64) << np.uint64(32)) | d).size == m
    assert s.max() < (1 << scale) and d.max() < (1 << scale)
    top = scale - 1
    sb, db = (s >> top) & 1, (d >> top) & 1
    freq = [np.mean((sb == i) & (db == j)) for i, j in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    for got, want in zip(freq, inputs.RMAT_ABCD):
        assert abs(got - want) < 0.03
    deg = np.bincount(s, minlength=1 << scale)
    assert deg.max() > 20 * deg.mean()      # hub skew


def test_scatter_ids_is_injective_relabelling():
    s, d = inputs.rmat(9, 400, *inputs.RMAT_ABCD, seed=6)
    s2, d2 = inputs.scatter_ids(s, d, 22, seed=6)
    assert s2.max() < (1 << 22) and d2.max() < (1 << 22)
    old = np.concatenate([s, d])
    new = np.concatenate([s2, d2])
    pairs = set(zip(old.tolist(), new.tolist()))
    assert len({o for o, _ in pairs}) == len(pairs) == len({n for _, n in pairs})


def test_shapes():
    s, d = inputs.grid_dag(3)
    assert s.size == 12
    s, d = inputs.binary_tree(3)
    assert s.size == 14 and np.all((d - 1) // 2 == s)
    s, d = inputs.cycle(4)
    assert d.tolist() == [1, 2, 3, 0]


def test_er_batch_layout():
    b = inputs.er_batch(16, seed=4)
    assert b.num == 16 and b.offsets[0] == 0 and b.offsets[-1] == b.src.size
    for i in range(b.num):
        s, d = b.instance(i)
        assert 256 <= b.n[i] <= 65536
        assert 0.5 * b.n[i] - 1 <= s.size <= 0.95 * b.n[i] + 1
        assert s.max(initial=0) < b.n[i] and d.max(initial=0) < b.n[i]


def test_broom_shape():
    s, d = inputs.broom(3, 4, 5)
    assert s.dtype == np.uint32 and d.dtype == np.uint32
    e = set(zip(s.tolist(), d.tolist()))
    assert len(e) == len(s) == 3 + 4 + 4 * 5
    assert {(0, 1), (1, 2), (2, 3)} <= e
    assert all((3, m) in e for m in range(4, 8))
    assert all((m, t) in e for m in range(4, 8) for t in range(8, 13))
