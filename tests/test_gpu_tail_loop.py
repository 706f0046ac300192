"""The default loop's tail loop: the fixpoint's tail run by one block in one launch,
against the oracle.

Once the delta and an iteration's candidates fit one block, a single workgroup loops over
whole iterations (join, sort, dedup + difference, merge into a run held in LDS) and a
multi-block launch folds that run into Full after it.  Results, iteration counts, every
delta size and the candidate totals must equal the oracle's, at small sizes and at the full
sizes of the stored summaries; the tail launch must have run where the sizes allow it.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2607_17571_amd import inputs
from paper_2607_17571_amd import wg
from tests.gpu_util import assert_same, digest, run
from tests.test_gpu_batch import _golden_batch, check_instances, run_batch

pytestmark = pytest.mark.gpu

NO_TAIL = wg.WG_NO_TAIL_LOOP
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fixpoints.json")))


def timed(**kw):
    kw["flags"] = kw.get("flags", 0) | wg.WG_STAGE_TIMING
    return wg.make_options(**kw)


TC_GRAPHS = {
    "chain200": lambda: inputs.chain(200),
    "cycle50": lambda: inputs.cycle(50),
    "grid12": lambda: inputs.grid_dag(12),
    "complete40": lambda: inputs.complete_dag(40),
    "star300": lambda: inputs.out_star(300),
    "er2000": lambda: inputs.erdos_renyi(2000, 1900, seed=2),
    "er300": lambda: inputs.erdos_renyi(300, 280, seed=1),
    "rmat11": lambda: inputs.rmat(11, 1800, *inputs.RMAT_ABCD, seed=9),
    "rmat12": lambda: inputs.rmat(12, 3600, *inputs.RMAT_ABCD, seed=4),
    "wide_ids": lambda: inputs.scatter_ids(*inputs.rmat(10, 900, *inputs.RMAT_ABCD, seed=4), 30, seed=5),
    "layers": lambda: inputs.layers_and_intree(3, 18, 5, 4, 30),
}


# graphs whose last iterations fit one block (the layered graph's joins stay above it)
TAIL_RUNS = {"chain200", "cycle50", "er2000", "er300", "grid12"}


@pytest.mark.parametrize("name", sorted(TC_GRAPHS))
def test_tc(engine, name):
    src, dst = TC_GRAPHS[name]()
    ref = oracle.tc(src, dst)
    s, d, st = run(engine, "tc", src, dst, timed())
    assert_same(s, d, st, ref)
    if name in TAIL_RUNS:
        assert st["stage_launches"]["tail_loop"] > 0, "the tail loop never ran"


@pytest.mark.parametrize("seed,n,m", [(1, 300, 280), (2, 2000, 1900), (3, 20000, 18000), (7, 50, 60)])
def test_sg(engine, seed, n, m):
    src, dst = inputs.erdos_renyi(n, m, seed=seed)
    ref = oracle.sg(src, dst)
    s, d, st = run(engine, "sg", src, dst, timed())
    assert_same(s, d, st, ref)


def test_sg_rmat_and_irreflexive(engine):
    src, dst = inputs.rmat(10, 900, *inputs.RMAT_ABCD, seed=3)
    s, d, st = run(engine, "sg", src, dst, timed())
    assert_same(s, d, st, oracle.sg(src, dst))
    s, d, st = run(engine, "sg", src, dst, timed(flags=wg.WG_SG_IRREFLEXIVE))
    ref = oracle.sg(src, dst, irreflexive=True)
    np.testing.assert_array_equal(s, ref.src)
    np.testing.assert_array_equal(d, ref.dst)


def test_long_chain_many_launches(engine):
    """1,200 iterations: the tail launches stop at their record bound and at a full run T
    (about a thousand new tuples per iteration), and each fold hands the next one a longer B."""
    src, dst = inputs.chain(1200)
    ref = oracle.tc(src, dst)
    s, d, st = run(engine, "tc", src, dst, timed())
    assert_same(s, d, st, ref)
    assert st["stage_launches"]["tail_loop"] > 10


@pytest.mark.parametrize("opts", [
    dict(), dict(flags=wg.WG_ITER_GRAPH), dict(flags=wg.WG_NO_SPECULATION), dict(batch_k=1),
    dict(radix_field_bits=32), dict(flags=wg.WG_SPARSE_INDEX), dict(flags=wg.WG_LSD_SORT),
    # variants that keep the multi-block launches (the tail loop is not used with them)
    dict(flags=wg.WG_UNFUSED_DEDUP), dict(flags=wg.WG_JOIN_HASH), dict(flags=wg.WG_JOIN_HASH_ROWS),
])
def test_with_other_options(engine, opts):
    src, dst = inputs.rmat(11, 1800, *inputs.RMAT_ABCD, seed=9)
    s, d, st = run(engine, "tc", src, dst, wg.make_options(**opts))
    assert_same(s, d, st, oracle.tc(src, dst))


@pytest.mark.parametrize("at", [1, 3, 6, 10, 11])
def test_forced_overflow(engine, at):
    """The overflow hook's iteration goes back to the multi-block path, which reports it."""
    src, dst = inputs.rmat(11, 1800, *inputs.RMAT_ABCD, seed=9)
    s, d, st = run(engine, "tc", src, dst, wg.make_options(force_overflow_at_iter=at))
    assert_same(s, d, st, oracle.tc(src, dst))
    assert st["resumes"] >= 1


def test_iteration_limit(engine):
    a, b = inputs.chain(100)
    with pytest.raises(wg.WgError) as ei:
        run(engine, "tc", a, b, wg.make_options(max_iterations=40))
    assert ei.value.status == wg.WG_ERR_ITER_LIMIT
    ref = oracle.tc(a, b)
    s, d, st = run(engine, "tc", a, b, wg.make_options(max_iterations=ref.iterations))
    assert_same(s, d, st, ref)


def test_empty_and_tiny(engine):
    for src, dst in [(np.zeros(0, np.uint32), np.zeros(0, np.uint32)), (np.array([3], np.uint32),
                                                                         np.array([3], np.uint32)),
                     (np.array([0, 1], np.uint32), np.array([1, 2], np.uint32))]:
        for q, fn in (("tc", oracle.tc), ("sg", oracle.sg)):
            s, d, st = run(engine, q, src, dst, timed())
            assert_same(s, d, st, fn(src, dst))


def test_alternating_with_other_loops(engine):
    """Tail-loop solves between solves of other loop modes and sizes on one engine."""
    cases = [("tc", inputs.chain(300)), ("sg", inputs.erdos_renyi(2000, 1900, seed=2)),
             ("tc", inputs.rmat(12, 3600, *inputs.RMAT_ABCD, seed=4))]
    for _ in range(2):
        for q, (src, dst) in cases:
            ref = oracle.tc(src, dst) if q == "tc" else oracle.sg(src, dst)
            for opts in (wg.make_options(), wg.make_options(flags=NO_TAIL), wg.make_options(),
                         wg.make_options(loop_mode=wg.WG_LOOP_HOST)):
                s, d, st = run(engine, q, src, dst, opts)
                assert_same(s, d, st, ref)


@pytest.mark.parametrize("name", ["tc_er_2000", "tc_rmat_s15", "tc_rmat_s16", "tc_rmat_s15_ids24",
                                  "sg_er_500k", "tc_grid_100"])
def test_full_size_without_tail_loop(engine, name):
    """The multi-block launches alone (the tail loop is the default's; the default runs
    against these summaries with the other full-size tests)."""
    g = GOLDEN[name]
    w = inputs.workload(name)
    s, d, st = run(engine, w.query, w.src, w.dst, wg.make_options(flags=NO_TAIL))
    assert s.size == g["size"]
    assert st["iterations"] == g["iterations"]
    assert st["delta_sizes"] == g["delta_sizes"]
    assert st["join_candidates"] == g["candidates"]
    assert digest(s, d) == g["sha256"]


def test_batches(engine):
    b = inputs.er_batch(40, seed=14, n_lo=16, n_hi=2000)
    refs = oracle.tc_batch(b.src, b.dst, b.offsets)
    s, d, offs, st = run_batch(engine, "tc", b.src, b.dst, b.offsets, timed())
    check_instances(s, d, offs, refs, range(b.num))
    assert st["stage_launches"]["tail_loop"] > 0
    refs = oracle.sg_batch(b.src, b.dst, b.offsets)
    s, d, offs, st = run_batch(engine, "sg", b.src, b.dst, b.offsets, timed())
    check_instances(s, d, offs, refs, range(b.num))


@pytest.mark.parametrize("name", ["tc_batch_er_256", "sg_batch_er_256", "tc_batch_er_4096"])
def test_batch_without_tail_loop_against_golden(engine, name):
    _golden_batch(engine, name, [0, 1, 100, 255], wg.make_options(flags=NO_TAIL))
