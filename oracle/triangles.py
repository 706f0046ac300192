"""Plain CPU oracle for triangle counting.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run this
module: only the test suite and the benchmark's CPU baseline use it.  It shares no code
with the HIP path.

Section VI states triangle counting as the non-recursive rule

    triangle(a, b, c) <- edge(a, b), edge(b, c), edge(c, a)

evaluated as a single pass of the sorted-array join: every edge (a, b) probes the edge
relation by source for the edges (b, c), and each two-path (a, c) so found is kept when
the edge (c, a) exists.  The count is the number of bindings (a, b, c) over the set of
edges (duplicates collapse; a self-loop is an ordinary edge, so (a, a, a) counts once
for an edge (a, a), and a directed 3-cycle counts once per rotation).

Reading: the paper reports timings, not the count's convention; bindings of the rule as
written are counted.  That number equals trace(A^3) of the 0/1 adjacency matrix, which
the tests use as an independent check.
"""

from __future__ import annotations

import numpy as np

U64 = np.uint64


def triangles(src, dst) -> tuple[int, int]:
    """Return (number of bindings of the triangle rule, number of two-paths joined)."""
    src = np.asarray(src, dtype=U64)
    dst = np.asarray(dst, dtype=U64)
    E = np.unique((src << U64(32)) | dst)  # the edge set, sorted (src, dst)
    E_src = (E >> U64(32)).astype(U64)
    E_dst = (E & U64(0xFFFFFFFF)).astype(U64)
    # join edge(a, b) with edge(b, c): the rows of E whose source is b
    lo = np.searchsorted(E_src, E_dst, side="left")
    hi = np.searchsorted(E_src, E_dst, side="right")
    counts = (hi - lo).astype(np.int64)
    two_paths = int(counts.sum())
    if two_paths == 0:
        return 0, 0
    owner = np.repeat(np.arange(E.size), counts)           # the edge (a, b) of each two-path
    first = np.repeat(lo, counts)
    rank = np.arange(two_paths) - np.repeat(np.cumsum(counts) - counts, counts)
    a = E_src[owner]
    c = E_dst[first + rank]                                 # the edge (b, c)
    # keep the two-paths whose closing edge (c, a) exists
    closing = (c << U64(32)) | a
    pos = np.searchsorted(E, closing)
    pos = np.minimum(pos, E.size - 1)
    return int(np.count_nonzero(E[pos] == closing)), two_paths
