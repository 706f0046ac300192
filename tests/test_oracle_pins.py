"""Pins for the CPU oracle, checked against facts that do not come from the oracle.

* the paper's worked example (Section II, Figure 1), stored under tests/golden/;
* closed forms for chains, cycles, stars, complete DAGs, grid DAGs, binary trees
  and the diamond;
* brute force written independently of the oracle: naive Datalog evaluation over
  Python sets, all-pairs BFS distances (scipy.sparse.csgraph) for TC, and boolean
  matrix products for SG;
* invariants: sortedness, E inside TC, closure under one more join, SG symmetry,
  SG with the diagonal removed equal to SG with x != y on every rule.

The last test plants plausible mistakes in the oracle and checks that this battery
catches each of them.
"""

import json
import os
from collections import defaultdict

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings
from hypothesis import strategies as st
from scipy.sparse.csgraph import shortest_path

import oracle
from oracle import seminaive
from paper_2607_17571_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Independent brute force (shares nothing with oracle/).
# ---------------------------------------------------------------------------

def naive_tc(edges):
    """Naive evaluation over Python sets: T_j = T_{j-1} | T_{j-1} o E until no change.

    Returns (fixpoint set, rounds including the unproductive one, |T_j| per round).
    After round j, naive and semi-naive evaluation hold the same relation.
    """
    E = set(edges)
    succ = defaultdict(set)
    for x, y in E:
        succ[x].add(y)
    T = set(E)
    sizes = [len(T)]
    rounds = 0
    if not T:
        return T, 0, sizes
    while True:
        rounds += 1
        new = {(x, z) for (x, y) in T for z in succ[y]}
        T2 = T | new
        sizes.append(len(T2))
        if T2 == T:
            return T, rounds, sizes
        T = T2


def naive_sg(edges, strict=False):
    """Naive SG over sets; ``strict`` applies x != y to the recursive rule as well."""
    E = set(edges)
    children = defaultdict(set)
    for p, c in E:
        children[p].add(c)
    S = {(x, y) for p in children for x in children[p] for y in children[p] if x != y}
    sizes = [len(S)]
    rounds = 0
    if not S:
        return S, 0, sizes
    while True:
        rounds += 1
        new = {(x, y) for (a, b) in S for x in children[a] for y in children[b]
               if not (strict and x == y)}
        S2 = S | new
        sizes.append(len(S2))
        if S2 == S:
            return S, rounds, sizes
        S = S2


def bfs_tc(src, dst, n):
    """TC and per-iteration delta sizes from all-pairs BFS distances.

    delta+(x, y) = 1 + min over out-neighbours u of x of dist(u, y).  (x, y) is in
    TC iff delta+ is finite, and semi-naive iteration i discovers exactly the pairs
    with delta+ = i + 1.
    """
    A = sp.csr_matrix((np.ones(src.size), (src.astype(np.int64), dst.astype(np.int64))),
                      shape=(n, n))
    D = shortest_path(A, method="D", unweighted=True)
    P = np.full((n, n), np.inf)
    np.minimum.at(P, src.astype(np.int64), D[dst.astype(np.int64)])
    P += 1.0
    finite = np.isfinite(P)
    xs, ys = np.nonzero(finite)
    dist = P[finite].astype(np.int64)
    hist = np.bincount(dist)[1:] if dist.size else np.zeros(0, dtype=np.int64)
    return xs, ys, hist


def matrix_sg(src, dst, n):
    """SG by boolean matrices: M1 = (A^T A > 0) minus I;  S <- S | (A^T S A > 0) to a fixpoint."""
    A = sp.csr_matrix((np.ones(src.size, dtype=np.int64),
                       (src.astype(np.int64), dst.astype(np.int64))), shape=(n, n))
    A.data[:] = 1
    A.sum_duplicates()
    A.data[:] = 1
    At = A.T.tocsr()
    S = (At @ A)
    S.setdiag(0)
    S.eliminate_zeros()
    S = (S > 0).astype(np.int64)
    sizes = [S.nnz]
    rounds = 0
    if S.nnz == 0:
        return S, 0, sizes
    while True:
        rounds += 1
        step = (At @ S @ A > 0).astype(np.int64)
        S2 = ((S + step) > 0).astype(np.int64)
        sizes.append(S2.nnz)
        if S2.nnz == S.nnz:
            return S, rounds, sizes
        S = S2


def as_set(r):
    return set(zip(r.src.tolist(), r.dst.tolist()))


def strictly_sorted(r):
    k = (r.src.astype(np.uint64) << np.uint64(32)) | r.dst.astype(np.uint64)
    return bool(np.all(k[1:] > k[:-1]))


# ---------------------------------------------------------------------------
# The paper's worked example.
# ---------------------------------------------------------------------------

def test_worked_example_fig1():
    g = json.load(open(os.path.join(GOLDEN, "tc_chain_fig1.json")))
    vid = g["vertices"]
    src = np.array([vid[a] for a, _ in g["edges"]], dtype=np.uint32)
    dst = np.array([vid[b] for _, b in g["edges"]], dtype=np.uint32)
    r = oracle.tc(src, dst, trace=True)
    assert r.iterations == g["iterations"]
    assert r.full_sizes == g["full_sizes"]
    assert r.delta_sizes == [len(d) for d in g["deltas"]]
    for got, want in zip(r.deltas, g["deltas"]):
        s, d = seminaive.unpack(got)
        assert set(zip(s.tolist(), d.tolist())) == {(vid[a], vid[b]) for a, b in want}
    assert as_set(r) == {(vid[a], vid[b]) for a, b in g["fixpoint"]}
    assert strictly_sorted(r)


# ---------------------------------------------------------------------------
# Closed forms.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 7, 40])
def test_chain_closed_form(n):
    r = oracle.tc(*inputs.chain(n))
    assert r.src.size == n * (n - 1) // 2
    assert r.iterations == n - 1
    assert r.delta_sizes == [n - 1 - i for i in range(n)]


@pytest.mark.parametrize("n", [1, 2, 5, 33])
def test_cycle_closed_form(n):
    r = oracle.tc(*inputs.cycle(n))
    assert r.src.size == n * n
    assert r.iterations == n
    assert r.delta_sizes == [n] * n + [0]


@pytest.mark.parametrize("d", [1, 2, 9])
def test_star_closed_form(d):
    t = oracle.tc(*inputs.out_star(d))
    assert t.src.size == d and t.iterations == 1
    s = oracle.sg(*inputs.out_star(d))
    assert s.src.size == d * (d - 1)
    assert s.iterations == (1 if d >= 2 else 0)


@pytest.mark.parametrize("n", [2, 6, 20])
def test_complete_dag_closed_form(n):
    r = oracle.tc(*inputs.complete_dag(n))
    assert r.src.size == n * (n - 1) // 2 and r.iterations == 1


@pytest.mark.parametrize("L", [2, 5, 12])
def test_grid_closed_form(L):
    r = oracle.tc(*inputs.grid_dag(L))
    assert r.src.size == (L * (L + 1) // 2) ** 2 - L * L
    assert r.iterations == 2 * (L - 1)


@pytest.mark.parametrize("h", [1, 2, 5])
def test_binary_tree_sg_closed_form(h):
    r = oracle.sg(*inputs.binary_tree(h))
    assert r.src.size == sum((1 << d) * ((1 << d) - 1) for d in range(1, h + 1))
    assert r.iterations == h
    assert np.all(r.src != r.dst)


def test_diamond_sg():
    lit = oracle.sg(*inputs.diamond())
    assert as_set(lit) == {(1, 2), (2, 1), (3, 3)} and lit.iterations == 2
    strict = oracle.sg(*inputs.diamond(), irreflexive=True)
    assert as_set(strict) == {(1, 2), (2, 1)}


def test_empty_inputs():
    e = np.empty(0, dtype=np.uint32)
    r = oracle.tc(e, e)
    assert r.src.size == 0 and r.iterations == 0 and r.delta_sizes == [0]
    r = oracle.sg(e, e)
    assert r.src.size == 0 and r.iterations == 0


def test_self_loop_and_duplicates_and_extreme_ids():
    top = 0xFFFFFFFF
    src = np.array([5, 5, top, 0, 0], dtype=np.uint32)
    dst = np.array([5, 5, 0, top, top], dtype=np.uint32)
    r = oracle.tc(src, dst)
    assert as_set(r) == {(5, 5), (top, 0), (0, top), (top, top), (0, 0)}
    assert strictly_sorted(r)


# ---------------------------------------------------------------------------
# Brute force on random graphs.
# ---------------------------------------------------------------------------

edges_strategy = st.lists(st.tuples(st.integers(0, 11), st.integers(0, 11)), max_size=40)


@settings(max_examples=150, deadline=None)
@given(edges_strategy)
def test_tc_matches_naive_sets(edges):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    r = oracle.tc(src, dst)
    T, rounds, sizes = naive_tc(edges)
    assert as_set(r) == T
    assert r.iterations == rounds
    assert r.full_sizes == sizes
    assert strictly_sorted(r)


@settings(max_examples=150, deadline=None)
@given(edges_strategy)
def test_sg_matches_naive_sets(edges):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    r = oracle.sg(src, dst)
    S, rounds, sizes = naive_sg(edges)
    assert as_set(r) == S
    assert r.iterations == rounds
    assert r.full_sizes == sizes
    strict, _, _ = naive_sg(edges, strict=True)
    assert as_set(oracle.sg(src, dst, irreflexive=True)) == strict


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_tc_matches_bfs_random(seed):
    n = 300
    src, dst = inputs.erdos_renyi(n, 330, seed=seed)
    r = oracle.tc(src, dst)
    xs, ys, hist = bfs_tc(src, dst, n)
    assert as_set(r) == set(zip(xs.tolist(), ys.tolist()))
    assert r.delta_sizes[:-1] == hist.tolist()
    assert r.iterations == hist.size


def test_tc_er_2000_config_matches_bfs():
    """The small TC configuration itself (ER n=2,000, m=1,900) by brute force."""
    w = inputs.workload("tc_er_2000")
    r = oracle.tc(w.src, w.dst)
    xs, ys, hist = bfs_tc(w.src, w.dst, 2000)
    assert r.src.size == xs.size
    got = (r.src.astype(np.int64) * 2000 + r.dst)
    want = np.sort(xs.astype(np.int64) * 2000 + ys)
    assert np.array_equal(got, want)
    assert r.delta_sizes[:-1] == hist.tolist() and r.iterations == hist.size


@pytest.mark.parametrize("seed,n,m", [(21, 200, 180), (22, 300, 280), (23, 120, 150)])
def test_sg_matches_matrix_random(seed, n, m):
    src, dst = inputs.erdos_renyi(n, m, seed=seed)
    r = oracle.sg(src, dst)
    S, rounds, sizes = matrix_sg(src, dst, n)
    S = S.tocoo()
    assert as_set(r) == set(zip(S.row.tolist(), S.col.tolist()))
    assert r.iterations == rounds
    assert r.full_sizes == sizes


def test_sg_matches_matrix_rmat():
    src, dst = inputs.rmat(8, 230, *inputs.RMAT_ABCD, seed=5)
    r = oracle.sg(src, dst)
    S, rounds, sizes = matrix_sg(src, dst, 256)
    S = S.tocoo()
    assert as_set(r) == set(zip(S.row.tolist(), S.col.tolist()))
    assert r.iterations == rounds


# ---------------------------------------------------------------------------
# Invariants at moderate size.
# ---------------------------------------------------------------------------

def test_tc_invariants_rmat():
    src, dst = inputs.rmat(11, 1800, *inputs.RMAT_ABCD, seed=7)
    r = oracle.tc(src, dst)
    assert strictly_sorted(r)
    T = seminaive.pack(r.src, r.dst)
    E = np.unique(seminaive.pack(src, dst))
    assert np.all(np.isin(E, T))                        # E inside TC
    E_src, E_dst = seminaive.unpack(E)
    once_more = seminaive.join_tc(T, E_src, E_dst)      # T o E inside T
    assert np.all(np.isin(once_more, T))
    assert r.full_sizes[-1] == r.src.size
    assert all(b - a == d for a, b, d in zip(r.full_sizes, r.full_sizes[1:], r.delta_sizes[1:]))


def test_sg_invariants_er():
    src, dst = inputs.erdos_renyi(5000, 4600, seed=9)
    r = oracle.sg(src, dst)
    assert strictly_sorted(r)
    fwd = set(zip(r.src.tolist(), r.dst.tolist()))
    assert fwd == {(y, x) for x, y in fwd}              # symmetric
    strict = oracle.sg(src, dst, irreflexive=True)
    edges = list(zip(src.tolist(), dst.tolist()))
    S_strict, _, _ = naive_sg(edges, strict=True)
    assert as_set(strict) == S_strict                  # literal minus diagonal == strict


# ---------------------------------------------------------------------------
# Batches: each instance's fixpoint, from its own slice of the edges and with local ids,
# pinned to BFS (TC) and boolean matrices (SG) per instance, never to the oracle's own
# single-instance path.  Empty instances sit first, in the middle and last.
# ---------------------------------------------------------------------------

def _ragged_batch(seed):
    rng = np.random.default_rng(seed)
    srcs, dsts, sizes, ns = [], [], [], []
    for i in range(14):
        n = int(rng.integers(2, 30))
        if i in (0, 6, 13):
            s = d = np.empty(0, np.uint32)
        else:
            m = int(rng.integers(1, min(2 * n, n * (n - 1)) + 1))
            s, d = inputs.erdos_renyi(n, m, seed=seed * 100 + i)
            if i % 4 == 1:  # a self-loop and a duplicate edge inside the instance
                s = np.concatenate([s, s[:1], s[:1]]).astype(np.uint32)
                d = np.concatenate([d, s[:1], d[:1]]).astype(np.uint32)
        srcs.append(s)
        dsts.append(d)
        sizes.append(s.size)
        ns.append(n)
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return np.concatenate(srcs), np.concatenate(dsts), offsets, ns


def _check_tc_batch(batch_fn):
    for seed in (1, 2, 3):
        src, dst, offs, ns = _ragged_batch(seed)
        res = batch_fn(src, dst, offs)
        assert len(res) == len(ns)
        for i, (r, n) in enumerate(zip(res, ns)):
            s, d = src[offs[i]:offs[i + 1]], dst[offs[i]:offs[i + 1]]
            xs, ys, hist = bfs_tc(s, d, n)
            assert as_set(r) == set(zip(xs.tolist(), ys.tolist())), (seed, i)
            assert strictly_sorted(r)
            # |Delta_i| = pairs first reached by a shortest positive walk of length i + 1
            assert r.delta_sizes == [int(h) for h in hist] + [0], (seed, i)
            assert r.iterations == hist.size


def _check_sg_batch(batch_fn):
    for seed in (4, 5):
        src, dst, offs, ns = _ragged_batch(seed)
        res = batch_fn(src, dst, offs)
        assert len(res) == len(ns)
        for i, (r, n) in enumerate(zip(res, ns)):
            s, d = src[offs[i]:offs[i + 1]], dst[offs[i]:offs[i + 1]]
            if s.size == 0:
                assert r.src.size == 0 and r.iterations == 0
                continue
            S, rounds, sizes = matrix_sg(s, d, n)
            xs, ys = S.nonzero()
            assert as_set(r) == set(zip(xs.tolist(), ys.tolist())), (seed, i)
            assert r.iterations == rounds and r.full_sizes == sizes


def test_tc_batch_matches_bfs_per_instance():
    _check_tc_batch(oracle.tc_batch)


def test_sg_batch_matches_matrices_per_instance():
    _check_sg_batch(oracle.sg_batch)


def _batch_shifted_slices(batch_src, batch_dst, offsets):
    """Planted mistake: every instance but the first starts one edge late."""
    return [oracle.tc(batch_src[int(offsets[i]) + (i > 0):int(offsets[i + 1])],
                      batch_dst[int(offsets[i]) + (i > 0):int(offsets[i + 1])])
            for i in range(len(offsets) - 1)]


def _batch_skips_empty(batch_src, batch_dst, offsets):
    """Planted mistake: empty instances are dropped from the list of results."""
    return [oracle.tc(batch_src[int(offsets[i]):int(offsets[i + 1])],
                      batch_dst[int(offsets[i]):int(offsets[i + 1])])
            for i in range(len(offsets) - 1) if offsets[i + 1] > offsets[i]]


@pytest.mark.parametrize("mistake", [_batch_shifted_slices, _batch_skips_empty])
def test_batch_pin_catches_planted_mistakes(mistake):
    with pytest.raises(AssertionError):
        _check_tc_batch(mistake)


# ---------------------------------------------------------------------------
# Planted mistakes must be caught by the pins above.
# ---------------------------------------------------------------------------

def _battery():
    """A fast subset of the pins; returns the number that fail (raising counts as failing)."""
    failures = 0
    checks = []
    g = json.load(open(os.path.join(GOLDEN, "tc_chain_fig1.json")))

    def fig1():
        vid = g["vertices"]
        src = np.array([vid[a] for a, _ in g["edges"]], dtype=np.uint32)
        dst = np.array([vid[b] for _, b in g["edges"]], dtype=np.uint32)
        r = oracle.tc(src, dst, max_iterations=20)
        assert r.iterations == g["iterations"] and r.full_sizes == g["full_sizes"]
    checks.append(fig1)

    def random_tc():
        for seed in range(5):
            src, dst = inputs.erdos_renyi(12, 20, seed=100 + seed)
            r = oracle.tc(src, dst, max_iterations=200)
            T, rounds, sizes = naive_tc(list(zip(src.tolist(), dst.tolist())))
            assert as_set(r) == T and r.full_sizes == sizes
    checks.append(random_tc)

    def random_sg():
        for seed in range(5):
            src, dst = inputs.erdos_renyi(12, 22, seed=200 + seed)
            r = oracle.sg(src, dst, max_iterations=200)
            S, rounds, sizes = naive_sg(list(zip(src.tolist(), dst.tolist())))
            assert as_set(r) == S and r.full_sizes == sizes
    checks.append(random_sg)

    def trees():
        r = oracle.sg(*inputs.binary_tree(3), max_iterations=50)
        assert r.src.size == 2 + 12 + 56 and r.iterations == 3
        d = oracle.sg(*inputs.diamond(), max_iterations=50)
        assert as_set(d) == {(1, 2), (2, 1), (3, 3)}
    checks.append(trees)

    for c in checks:
        try:
            c()
        except Exception:  # noqa: BLE001 - any failure counts
            failures += 1
    return failures


def _mut_join_on_src(delta, E_src, E_dst):
    a, b = seminaive.unpack(delta)
    lo, hi = seminaive.edge_range(E_src, a)
    owner, rank = seminaive._expand(hi - lo)
    return seminaive.pack(a[owner], E_dst[lo[owner] + rank])


def _mut_join_wrong_head(delta, E_src, E_dst):
    a, b = seminaive.unpack(delta)
    lo, hi = seminaive.edge_range(E_src, b)
    owner, rank = seminaive._expand(hi - lo)
    return seminaive.pack(b[owner], E_dst[lo[owner] + rank])


def _mut_sg_wrong_range(delta, E_src, E_dst):
    a, b = seminaive.unpack(delta)
    lo_a, hi_a = seminaive.edge_range(E_src, a)
    lo_b, hi_b = seminaive.edge_range(E_src, b)
    len_a, len_b = hi_a - lo_a, hi_b - lo_b
    owner, rank = seminaive._expand(len_a * len_b)
    x = E_dst[lo_a[owner] + rank // len_b[owner]]
    y = E_dst[np.minimum(lo_a[owner] + rank % len_b[owner], E_dst.size - 1)]
    return seminaive.pack(x, y)


def _mut_sg_base_no_filter(E_src, E_dst):
    parents = np.unique(E_src)
    lo, hi = seminaive.edge_range(E_src, parents)
    n = hi - lo
    owner, rank = seminaive._expand(n * n)
    return seminaive.pack(E_dst[lo[owner] + rank // n[owner]], E_dst[lo[owner] + rank % n[owner]])


MUTATIONS = {
    "join keyed on delta.src": ("join_tc", _mut_join_on_src),
    "join keeps the wrong head column": ("join_tc", _mut_join_wrong_head),
    "no set difference": ("set_difference", lambda S, full: S),
    "no dedup": ("sort_unique", lambda k: np.sort(k)),
    "merge drops the delta": ("merge", lambda full, delta: full),
    "edge range empty": ("edge_range", lambda E_src, v: (np.searchsorted(E_src, v, "left"),) * 2),
    "sg second factor from the wrong range": ("join_sg", _mut_sg_wrong_range),
    "sg base keeps x == y": ("sg_base", _mut_sg_base_no_filter),
}


def test_battery_passes_on_the_oracle():
    assert _battery() == 0


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(seminaive, attr, fn)
    assert _battery() > 0, f"planted mistake not caught: {name}"
