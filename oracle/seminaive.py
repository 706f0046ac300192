"""Plain CPU oracle for semi-naive TC and SG fixpoints.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run this
module: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path (no kernels, headers,
helpers or tables); both sides only read the same seeded inputs.

Everything is exact integer work on numpy arrays, single-threaded, written for a
reader to check against the paper by eye:

* a relation is a duplicate-free, ascending array of 64-bit keys ``(src << 32) | dst``
  -- lexicographic (src, dst) order on unsigned 32-bit ids (Section IV-A: base, delta
  and full relations are lexicographically sorted at every stage boundary);
* one semi-naive iteration is join -> sort -> dedup -> set difference -> merge
  (Section II, paragraph "Semi-Naive Evaluation", and Section II-A);
* the loop stops at the first empty delta.

Readings where the paper is silent (each is also listed in the design notes):

* the iteration count includes the final iteration whose delta is empty (the
  worked example of Section II takes three iterations on a four-vertex chain);
  an empty seed gives zero iterations;
* input edges form a multiset in any order; duplicates collapse, self-loops are
  ordinary edges;
* SG uses the rules ``SG(x,y) <- E(p,x), E(p,y), x != y`` (base) and
  ``SG(x,y) <- E(a,x), SG(a,b), E(b,y)`` (recursive), with E oriented parent ->
  child; the x != y filter applies to the base rule only.  ``irreflexive=True``
  drops (x,x) from the final relation.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

U32 = np.uint32
U64 = np.uint64
_LOW = U64(0xFFFFFFFF)


@dataclass
class Fixpoint:
    src: np.ndarray              # uint32, lexicographically sorted with dst
    dst: np.ndarray              # uint32
    iterations: int              # join rounds, including the one that yields the empty delta
    delta_sizes: list = field(default_factory=list)  # |Delta^0|, |Delta^1|, ..., |Delta^iterations|
    full_sizes: list = field(default_factory=list)   # |Full| after seeding and after each iteration
    candidates: int = 0          # join candidates summed over all iterations (with multiplicity)
    deltas: list = field(default_factory=list)       # Delta^i as key arrays, only when traced


def pack(src, dst) -> np.ndarray:
    """(src, dst) -> 64-bit keys whose numeric order is the lexicographic pair order."""
    return (np.asarray(src, dtype=U64) << U64(32)) | np.asarray(dst, dtype=U64)


def unpack(keys: np.ndarray):
    return (keys >> U64(32)).astype(U32), (keys & _LOW).astype(U32)


def sort_unique(keys: np.ndarray) -> np.ndarray:
    """Sort + deduplicate: a relation is a set (Section II)."""
    return np.unique(keys)


def edge_index(E: np.ndarray):
    """Split the sorted edge relation into its source column and destination column.

    E is sorted once and never modified, so all edges leaving vertex v occupy the
    contiguous range ``[lower_bound(E.src, v), upper_bound(E.src, v))`` (Section IV-A).
    """
    return unpack(E)


def edge_range(E_src: np.ndarray, v: np.ndarray):
    """Binary-search the source column for the contiguous range of each key in ``v``."""
    lo = np.searchsorted(E_src, v, side="left")
    hi = np.searchsorted(E_src, v, side="right")
    return lo.astype(np.int64), hi.astype(np.int64)


def _expand(counts: np.ndarray):
    """For a list of per-tuple counts, return (tuple index, rank within tuple) of every output."""
    owner = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    starts = np.cumsum(counts) - counts
    rank = np.arange(owner.size, dtype=np.int64) - starts[owner]
    return owner, rank


def join_tc(delta: np.ndarray, E_src: np.ndarray, E_dst: np.ndarray) -> np.ndarray:
    """T(x,z) <- Delta(x,y), E(y,z)  (Section II; binary-search join of Section IV-A).

    For each delta tuple (a, b) find the range of b in E.src and emit (a, E.dst[k])
    for every k in that range.  Candidates keep their multiplicity.
    """
    a, b = unpack(delta)
    lo, hi = edge_range(E_src, b)
    owner, rank = _expand(hi - lo)
    return pack(a[owner], E_dst[lo[owner] + rank])


def join_sg(delta: np.ndarray, E_src: np.ndarray, E_dst: np.ndarray) -> np.ndarray:
    """SG(x,y) <- E(a,x), SG(a,b), E(b,y)  (Section VI, same-generation).

    Each delta tuple (a, b) looks up two ranges in E -- children of a and children
    of b -- and emits their cross product (x, y).
    """
    a, b = unpack(delta)
    lo_a, hi_a = edge_range(E_src, a)
    lo_b, hi_b = edge_range(E_src, b)
    len_a, len_b = hi_a - lo_a, hi_b - lo_b
    owner, rank = _expand(len_a * len_b)
    x = E_dst[lo_a[owner] + rank // len_b[owner]]
    y = E_dst[lo_b[owner] + rank % len_b[owner]]
    return pack(x, y)


def sg_base(E_src: np.ndarray, E_dst: np.ndarray) -> np.ndarray:
    """SG(x,y) <- E(p,x), E(p,y), x != y: ordered pairs of distinct children of one parent."""
    parents = np.unique(E_src)
    lo, hi = edge_range(E_src, parents)
    n = hi - lo
    owner, rank = _expand(n * n)
    x = E_dst[lo[owner] + rank // n[owner]]
    y = E_dst[lo[owner] + rank % n[owner]]
    keep = x != y
    return pack(x[keep], y[keep])


def set_difference(S: np.ndarray, full: np.ndarray) -> np.ndarray:
    """Tuples of the sorted set S that are absent from the sorted set ``full``."""
    return np.setdiff1d(S, full, assume_unique=True)


def merge(full: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """Merge two disjoint sorted sets into one sorted set of size |full| + |delta| (Section IV-C)."""
    out = np.concatenate([full, delta])
    out.sort(kind="stable")
    return out


def _fixpoint(seed: np.ndarray, E: np.ndarray, join, max_iterations=None,
              trace: bool = False) -> Fixpoint:
    """Semi-naive loop (Section II, paragraph "Semi-Naive Evaluation").

    Delta^0 = Full = seed.  Iteration i joins Delta^{i-1} against E, removes duplicate
    candidates and those already in Full; the survivors are Delta^i and are merged
    into Full.  Evaluation stops when Delta^i is empty.
    """
    E_src, E_dst = edge_index(E)
    full = seed
    delta = seed
    delta_sizes = [int(delta.size)]
    full_sizes = [int(full.size)]
    iterations = 0
    candidates = 0
    deltas = [delta] if trace else []
    while delta.size > 0:
        if max_iterations is not None and iterations >= max_iterations:
            raise RuntimeError("iteration limit reached")
        iterations += 1
        cand = join(delta, E_src, E_dst)
        candidates += int(cand.size)
        fresh = set_difference(sort_unique(cand), full)
        full = merge(full, fresh)
        delta = fresh
        delta_sizes.append(int(delta.size))
        full_sizes.append(int(full.size))
        if trace:
            deltas.append(delta)
    s, d = unpack(full)
    return Fixpoint(s, d, iterations, delta_sizes, full_sizes, candidates, deltas)


def tc(src, dst, max_iterations=None, trace: bool = False) -> Fixpoint:
    """Transitive closure: T(x,y) <- E(x,y);  T(x,z) <- T(x,y), E(y,z)  (Section II)."""
    E = sort_unique(pack(src, dst))
    return _fixpoint(E, E, join_tc, max_iterations, trace)


def sg(src, dst, irreflexive: bool = False, max_iterations=None,
       trace: bool = False) -> Fixpoint:
    """Same generation with the base rule seeding Delta^0 = Full (Section VI)."""
    E = sort_unique(pack(src, dst))
    E_src, E_dst = edge_index(E)
    base = sort_unique(sg_base(E_src, E_dst))
    out = _fixpoint(base, E, join_sg, max_iterations, trace)
    if irreflexive:
        keep = out.src != out.dst
        out.src, out.dst = out.src[keep], out.dst[keep]
    return out


def tc_batch(batch_src, batch_dst, offsets):
    """Independent TC fixpoints of instances laid out back to back (ids local per instance)."""
    return [tc(batch_src[int(offsets[i]):int(offsets[i + 1])],
               batch_dst[int(offsets[i]):int(offsets[i + 1])])
            for i in range(len(offsets) - 1)]


def sg_batch(batch_src, batch_dst, offsets, irreflexive: bool = False):
    return [sg(batch_src[int(offsets[i]):int(offsets[i + 1])],
               batch_dst[int(offsets[i]):int(offsets[i + 1])], irreflexive)
            for i in range(len(offsets) - 1)]
