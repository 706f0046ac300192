"""Seeded synthetic edge relations shared by the GPU path, its tests and the oracle.

This module only draws and lays out input graphs: it holds none of the fixpoint
arithmetic (no join, sort-into-relation, dedup, difference or merge).  Every
generator is deterministic for a given seed (numpy PCG64 streams) and returns two
``uint32`` numpy arrays ``(src, dst)`` in draw order; the engine accepts any order
and duplicates, so nothing here sorts for it.

The paper evaluates on SNAP / SuiteSparse graphs (Section VII, "Datasets") that are
not available; the seeded Erdos-Renyi and R-MAT graphs below stand in for them with
the shapes the workloads name: uniform sparse graphs, skewed power-law graphs with
hub vertices (the skew of Section III-A), long-fixpoint meshes (grid DAGs), and
family trees for same-generation (Section VI).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

U32 = np.uint32
U64 = np.uint64


def _rng(*seed_words: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed_words))))


def _take_distinct(draw, m: int, rng: np.random.Generator):
    """Draw batches of (src, dst) until exactly ``m`` distinct non-loop pairs exist.

    ``draw(k)`` returns two uint64 arrays of ``k`` candidate endpoints.  Pairs are kept
    in order of first appearance, so the output is a prefix-stable function of the
    random stream.
    """
    keys = np.empty(0, dtype=U64)
    have = 0
    while have < m:
        k = int((m - have) * 1.25) + 64
        s, d = draw(k)
        keep = s != d
        new = (s[keep] << U64(32)) | d[keep]
        keys = np.concatenate([keys, new])
        _, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)]
        have = keys.size
    keys = keys[:m]
    return (keys >> U64(32)).astype(U32), (keys & U64(0xFFFFFFFF)).astype(U32)


def erdos_renyi(n: int, m: int, seed: int):
    """Directed G(n, m): endpoints uniform in [0, n), self-loops and duplicates redrawn."""
    if n < 2 and m > 0:
        raise ValueError("need n >= 2 for a loop-free edge")
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of loop-free ordered pairs")
    rng = _rng(0x45524, seed, n, m)

    def draw(k):
        return (rng.integers(0, n, k, dtype=U64), rng.integers(0, n, k, dtype=U64))

    return _take_distinct(draw, m, rng)


def rmat(scale: int, m: int, a: float, b: float, c: float, d: float, seed: int):
    """R-MAT graph on 2**scale vertices.

    At every bit level (most significant first) an edge picks quadrant a=(0,0),
    b=(0,1), c=(1,0) or d=(1,1) for (src bit, dst bit).  No noise and no vertex
    permutation, so low ids are the hubs.
    """
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("quadrant probabilities must sum to 1")
    rng = _rng(0x524D4154, seed, scale, m)
    cut1, cut2, cut3 = a, a + b, a + b + c

    def draw(k):
        s = np.zeros(k, dtype=U64)
        t = np.zeros(k, dtype=U64)
        for level in range(scale):
            u = rng.random(k)
            sbit = (u >= cut2).astype(U64)
            tbit = (((u >= cut1) & (u < cut2)) | (u >= cut3)).astype(U64)
            shift = U64(scale - 1 - level)
            s |= sbit << shift
            t |= tbit << shift
        return s, t

    return _take_distinct(draw, m, rng)


def scatter_ids(src, dst, id_bits: int, seed: int):
    """Relabel vertex ids through a seeded injective map into [0, 2**id_bits).

    Used to exercise wide id spaces (24- and 32-bit radix fields) on graphs whose
    structure is otherwise unchanged.
    """
    ids = np.unique(np.concatenate([src, dst]))
    rng = _rng(0x5343, seed, id_bits)
    space = 1 << id_bits
    picked = np.empty(0, dtype=U64)
    while picked.size < ids.size:
        more = rng.integers(0, space, ids.size * 2 + 16, dtype=U64)
        picked = np.concatenate([picked, more])
        _, first = np.unique(picked, return_index=True)
        picked = picked[np.sort(first)]
    new = picked[: ids.size].astype(U32)
    return new[np.searchsorted(ids, src)], new[np.searchsorted(ids, dst)]


# ---------------------------------------------------------------------------
# Small structured shapes with known closures (used as test inputs).
# ---------------------------------------------------------------------------

def chain(n: int):
    """Path 0 -> 1 -> ... -> n-1."""
    v = np.arange(max(n - 1, 0), dtype=U32)
    return v, v + U32(1)


def cycle(n: int):
    """Directed cycle 0 -> 1 -> ... -> n-1 -> 0."""
    v = np.arange(n, dtype=U32)
    return v, ((v + U32(1)) % U32(n)).astype(U32)


def out_star(d: int, centre: int = 0):
    """One centre with ``d`` leaf children (ids centre+1 .. centre+d)."""
    leaves = np.arange(centre + 1, centre + 1 + d, dtype=U32)
    return np.full(d, centre, dtype=U32), leaves


def complete_dag(n: int):
    """Edges i -> j for every i < j."""
    i, j = np.triu_indices(n, k=1)
    return i.astype(U32), j.astype(U32)


def grid_dag(L: int):
    """L x L grid with edges to the right and downwards; vertex (r, c) has id r*L + c."""
    r, c = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    v = (r * L + c).ravel()
    right = (c < L - 1).ravel()
    down = (r < L - 1).ravel()
    src = np.concatenate([v[right], v[down]])
    dst = np.concatenate([v[right] + 1, v[down] + L])
    return src.astype(U32), dst.astype(U32)


def binary_tree(depth: int):
    """Complete binary tree, root 0, children of v are 2v+1 and 2v+2, leaves at ``depth``."""
    nodes = (1 << (depth + 1)) - 1
    child = np.arange(1, nodes, dtype=U32)
    return ((child - U32(1)) // U32(2)).astype(U32), child


def broom(K: int, M: int, T: int):
    """A chain 0 -> 1 -> ... -> K, then K -> every one of M middle vertices and every
    middle vertex -> every one of T targets (ids K+1 .. K+M, then K+M+1 .. K+M+T)."""
    chain_s = np.arange(0, K, dtype=U32)
    mids = np.arange(K + 1, K + 1 + M, dtype=U32)
    tgts = np.arange(K + 1 + M, K + 1 + M + T, dtype=U32)
    src = np.concatenate([chain_s, np.full(M, K, dtype=U32), np.repeat(mids, T)])
    dst = np.concatenate([chain_s + U32(1), mids, np.tile(tgts, M)])
    return src.astype(U32), dst.astype(U32)


def diamond():
    """p -> a, p -> b, a -> x, b -> x with p=0, a=1, b=2, x=3."""
    return np.array([0, 0, 1, 2], dtype=U32), np.array([1, 2, 3, 3], dtype=U32)


def layers_and_intree(K: int, W: int, H: int, F: int, D: int):
    """Two components whose per-iteration join sizes first shrink, then jump.

    (1) K + 1 layers of W vertices, every vertex of layer k pointing to every vertex of
    layer k + 1 (ids 0 .. (K+1)W-1); (2) an F-ary in-tree of depth H whose edges point
    towards its root r, and r pointing to D fresh leaves.  Under transitive closure the
    layered part's joins shrink each iteration and end after K of them, while the paths
    reaching r multiply by F per iteration, each joining with r's D out-edges.
    """
    src, dst = [], []
    for k in range(K):
        for a in range(W):
            for b in range(W):
                src.append(k * W + a)
                dst.append((k + 1) * W + b)
    root = (K + 1) * W
    nxt = root + 1
    level = [root]
    for _ in range(H):
        new = []
        for p in level:
            for _ in range(F):
                src.append(nxt)
                dst.append(p)
                new.append(nxt)
                nxt += 1
        level = new
    for _ in range(D):
        src.append(root)
        dst.append(nxt)
        nxt += 1
    return np.array(src, dtype=U32), np.array(dst, dtype=U32)


# ---------------------------------------------------------------------------
# Workload recipes (the shapes the benchmarks and parity tests run).
# ---------------------------------------------------------------------------

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


@dataclass(frozen=True)
class Workload:
    name: str
    query: str  # "tc" or "sg"
    src: np.ndarray
    dst: np.ndarray


def workload(name: str) -> Workload:
    """Named synthetic workloads.

    tc_er_2000         directed ER, n=2,000, m=1,900, seed 1
    tc_rmat_s15        R-MAT scale 15, m=29,491 (0.9 * 2**15), seed 2
    tc_rmat_s16        R-MAT scale 16, m=58,982 (0.9 * 2**16), seed 2
    tc_rmat_s15_ids24  tc_rmat_s15 with ids scattered into [0, 2**22)
    tc_rmat_s22        R-MAT scale 22, m=3,800,000 (closure does not fit one GPU)
    sg_er_500k         directed ER, n=500,000, m=450,000, seed 3
    tc_grid_100        100 x 100 grid DAG (198-iteration fixpoint)
    """
    if name == "tc_er_2000":
        s, d = erdos_renyi(2000, 1900, seed=1)
        return Workload(name, "tc", s, d)
    if name == "tc_rmat_s15":
        s, d = rmat(15, 29491, *RMAT_ABCD, seed=2)
        return Workload(name, "tc", s, d)
    if name == "tc_rmat_s16":
        s, d = rmat(16, 58982, *RMAT_ABCD, seed=2)
        return Workload(name, "tc", s, d)
    if name == "tc_rmat_s15_ids24":
        s, d = rmat(15, 29491, *RMAT_ABCD, seed=2)
        s, d = scatter_ids(s, d, 22, seed=2)
        return Workload(name, "tc", s, d)
    if name == "tc_rmat_s22":
        s, d = rmat(22, 3_800_000, *RMAT_ABCD, seed=2)
        return Workload(name, "tc", s, d)
    if name == "sg_er_500k":
        s, d = erdos_renyi(500_000, 450_000, seed=3)
        return Workload(name, "sg", s, d)
    if name == "tc_grid_100":
        s, d = grid_dag(100)
        return Workload(name, "tc", s, d)
    raise KeyError(name)


@dataclass(frozen=True)
class Batch:
    """Many independent instances laid out back to back.

    ``offsets`` has ``num + 1`` entries; instance ``i`` owns edges
    ``offsets[i]:offsets[i+1]`` and its vertex ids are local to it (0 .. n_i - 1).
    """
    src: np.ndarray
    dst: np.ndarray
    offsets: np.ndarray
    n: np.ndarray

    @property
    def num(self) -> int:
        return int(self.offsets.size - 1)

    def instance(self, i: int):
        lo, hi = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.src[lo:hi], self.dst[lo:hi]


def er_batch(num: int, seed: int, n_lo: int = 256, n_hi: int = 65536,
             deg_lo: float = 0.5, deg_hi: float = 0.95) -> Batch:
    """``num`` ER instances, n log-uniform in [n_lo, n_hi], mean out-degree uniform in
    [deg_lo, deg_hi], m = round(degree * n)."""
    rng = _rng(0x4241, seed, num)
    n = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), num))).astype(np.int64)
    deg = rng.uniform(deg_lo, deg_hi, num)
    m = np.rint(deg * n).astype(np.int64)
    srcs, dsts = [], []
    for i in range(num):
        s, d = erdos_renyi(int(n[i]), int(m[i]), seed=seed * 1_000_003 + i)
        srcs.append(s)
        dsts.append(d)
    offsets = np.zeros(num + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(m).astype(np.uint64)
    return Batch(np.concatenate(srcs) if srcs else np.empty(0, U32),
                 np.concatenate(dsts) if dsts else np.empty(0, U32), offsets, n)


def batch_workload(name: str) -> tuple[str, Batch]:
    """Named batched workloads: (query, batch).

    tc_batch_er_4096   4,096 ER instances, n log-uniform in [256, 65,536], mean
                       out-degree uniform in [0.5, 0.95], seed 4
    tc_batch_er_256    the same recipe with 256 instances, seed 6 (a smaller batch)
    sg_batch_er_256    SG over 256 instances, n in [64, 4,096], seed 7
    """
    if name == "tc_batch_er_4096":
        return "tc", er_batch(4096, seed=4)
    if name == "tc_batch_er_256":
        return "tc", er_batch(256, seed=6)
    if name == "sg_batch_er_256":
        return "sg", er_batch(256, seed=7, n_lo=64, n_hi=4096)
    raise KeyError(name)


@dataclass(frozen=True)
class Request:
    """One served request: a TC or SG query on a seeded graph."""
    query: str
    kind: str  # "er" or "rmat"
    n: int
    src: np.ndarray
    dst: np.ndarray


def served_requests(num: int, seed: int, n_lo: int = 1000, n_hi: int = 1_000_000,
                    rmat_max_scale: int = 15, tc_share: float = 0.7) -> list:
    """The served mix: 70% TC / 30% SG, half ER and half R-MAT (0.57, 0.19, 0.19, 0.05),
    n log-uniform in [n_lo, n_hi], mean out-degree uniform in [0.5, 0.95].  R-MAT graphs
    take scale round(log2 n) capped at rmat_max_scale (larger R-MAT closures do not fit
    one device) and at least 4; m = round(degree * 2^scale)."""
    rng = _rng(0x5352, seed, num)
    out = []
    for i in range(num):
        query = "tc" if rng.random() < tc_share else "sg"
        kind = "er" if rng.random() < 0.5 else "rmat"
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        deg = float(rng.uniform(0.5, 0.95))
        sub = seed * 1_000_003 + i
        if kind == "er":
            s, d = erdos_renyi(n, max(1, int(round(deg * n))), seed=sub)
        else:
            scale = min(rmat_max_scale, max(4, int(round(math.log2(n)))))
            n = 1 << scale
            s, d = rmat(scale, max(1, int(round(deg * n))), *RMAT_ABCD, seed=sub)
        out.append(Request(query, kind, n, s, d))
    return out
