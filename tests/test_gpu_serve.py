"""Request server (wg_server_*): continuous batching keeps every result exact.

Each served result must be byte-identical to the same request solved alone through
wg_tc / wg_sg, and to the oracle.  Admission under a tight memory budget, requeueing,
rejection of an oversize request, cancellation and host-pointer inputs are covered.
"""

import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2607_17571_amd import inputs
from paper_2607_17571_amd import wg
from tests.gpu_util import run as run_single
from tests.gpu_util import to_gpu

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fixpoints.json")))


def served(server, reqs, host=False):
    jobs = []
    for r in reqs:
        if host:
            jobs.append(server.submit(r.query, r.src, r.dst))
        else:
            jobs.append(server.submit(r.query, to_gpu(r.src), to_gpu(r.dst)))
    out = []
    for j in jobs:
        s, d, st, info = j.wait()
        out.append((s.cpu().numpy(), d.cpu().numpy(), st, info))
        j.close()
    return out


def test_alone_equals_in_mix(engine):
    reqs = inputs.served_requests(24, seed=21, n_lo=100, n_hi=3000)
    print(f"[gpu] serve mix of {len(reqs)}", flush=True, file=sys.stderr)
    srv = wg.Server(0, slots=4, mem_budget_bytes=8 << 30)
    try:
        mix = served(srv, reqs)
        stats = srv.stats()
    finally:
        srv.close()
    for r, (s, d, st, info) in zip(reqs, mix):
        a_s, a_d, a_st = run_single(engine, r.query, r.src, r.dst)
        np.testing.assert_array_equal(s, a_s)
        np.testing.assert_array_equal(d, a_d)
        assert st["iterations"] == a_st["iterations"]
        assert st["delta_sizes"] == a_st["delta_sizes"]
        ref = oracle.tc(r.src, r.dst) if r.query == "tc" else oracle.sg(r.src, r.dst)
        np.testing.assert_array_equal(s, ref.src)
        np.testing.assert_array_equal(d, ref.dst)
        assert info["phase"] == 2 and info["status"] == wg.WG_OK
        assert info["submit_ms"] <= info["start_ms"] <= info["end_ms"]
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["held_bytes"] == 0  # every result freed
    assert stats["max_running"] >= 2  # the requests did share the device


@pytest.mark.parametrize("hold_after_us", [1, 0xFFFFFFFF], ids=["hold-1us", "never-hold"])
def test_long_solve_hold_keeps_results(engine, hold_after_us):
    """The long-solve hold changes only when requests start: with a 1 us hold (every running
    solve holds back the queue: nearly one at a time) and with no hold, every result equals
    the request solved alone."""
    reqs = inputs.served_requests(12, seed=22, n_lo=100, n_hi=3000)
    print(f"[gpu] serve mix of {len(reqs)}, hold {hold_after_us} us", flush=True, file=sys.stderr)
    srv = wg.Server(0, slots=4, mem_budget_bytes=8 << 30, hold_after_us=hold_after_us)
    try:
        mix = served(srv, reqs)
        stats = srv.stats()
    finally:
        srv.close()
    for r, (s, d, st, info) in zip(reqs, mix):
        a_s, a_d, a_st = run_single(engine, r.query, r.src, r.dst)
        np.testing.assert_array_equal(s, a_s)
        np.testing.assert_array_equal(d, a_d)
        assert st["iterations"] == a_st["iterations"]
        assert info["phase"] == 2 and info["status"] == wg.WG_OK
    assert stats["completed"] == len(reqs) and stats["failed"] == 0


def test_tight_budget_requeues_and_rejects_oversize(engine):
    """A 320 MB budget: medium requests must share it; one request needs far more."""
    reqs = [inputs.Request("tc", "rmat", 1 << 12, *inputs.rmat(12, 3800, *inputs.RMAT_ABCD, seed=s))
            for s in (31, 32, 33)]
    reqs += [inputs.Request("sg", "rmat", 1 << 11, *inputs.rmat(11, 1900, *inputs.RMAT_ABCD, seed=34))]
    big = inputs.workload("tc_rmat_s15")
    print("[gpu] serve under a tight budget", flush=True, file=sys.stderr)
    srv = wg.Server(0, slots=3, mem_budget_bytes=320 << 20)
    try:
        jobs = [srv.submit(r.query, to_gpu(r.src), to_gpu(r.dst)) for r in reqs]
        jbig = srv.submit("tc", to_gpu(big.src), to_gpu(big.dst))
        results = [j.wait() for j in jobs]
        with pytest.raises(wg.WgError) as ei:
            jbig.wait()
        assert ei.value.status == wg.WG_ERR_CAPACITY
        stats = srv.stats()
        for j in jobs + [jbig]:
            j.close()
    finally:
        srv.close()
    for r, (s, d, st, info) in zip(reqs, results):
        ref = oracle.tc(r.src, r.dst) if r.query == "tc" else oracle.sg(r.src, r.dst)
        np.testing.assert_array_equal(s.cpu().numpy(), ref.src)
        np.testing.assert_array_equal(d.cpu().numpy(), ref.dst)
    assert stats["completed"] == len(reqs) and stats["failed"] == 1
    assert stats["requeued"] >= 1  # some solve outgrew its reservation and was queued again


def test_cancel_queued_request(engine):
    srv = wg.Server(0, slots=1, mem_budget_bytes=4 << 30)
    try:
        g = inputs.grid_dag(60)
        first = srv.submit("tc", to_gpu(g[0]), to_gpu(g[1]))  # keeps the only slot busy
        small = [srv.submit("tc", *map(to_gpu, inputs.chain(20 + k))) for k in range(4)]
        small[2].cancel()
        with pytest.raises(wg.WgError) as ei:
            small[2].wait()
        assert ei.value.status == wg.WG_ERR_CANCELLED
        first.wait()
        for k in (0, 1, 3):
            s, d, st, _ = small[k].wait()
            ref = oracle.tc(*inputs.chain(20 + k))
            np.testing.assert_array_equal(s.cpu().numpy(), ref.src)
        stats = srv.stats()
        for j in [first] + small:
            j.close()
    finally:
        srv.close()
    assert stats["cancelled"] == 1


def test_host_pointer_inputs_and_empty_request(engine):
    reqs = inputs.served_requests(6, seed=22, n_lo=50, n_hi=500)
    srv = wg.Server(0, slots=2, mem_budget_bytes=2 << 30)
    try:
        host = served(srv, reqs, host=True)
        e = srv.submit("tc", np.empty(0, np.uint32), np.empty(0, np.uint32))
        s, d, st, _ = e.wait()
        assert s.numel() == 0 and st["iterations"] == 0
        e.close()
    finally:
        srv.close()
    for r, (s, d, st, info) in zip(reqs, host):
        ref = oracle.tc(r.src, r.dst) if r.query == "tc" else oracle.sg(r.src, r.dst)
        np.testing.assert_array_equal(s, ref.src)
        np.testing.assert_array_equal(d, ref.dst)


def _sha(s, d):
    return hashlib.sha256(np.asarray(s, dtype="<u4").tobytes() + np.asarray(d, dtype="<u4").tobytes()).hexdigest()


def test_served_mix_full_size_against_golden(engine):
    """The served mix at its real sizes (120 requests, n log-uniform in [1k, 1M], R-MAT up to
    scale 15, 4 slots, the default budget): every result equals the oracle's stored record
    (size, iterations, sha256) and the same request solved alone, and solves overlapped."""
    import torch

    g = GOLDEN["served_mix_120_seed5"]["requests"]
    reqs = inputs.served_requests(len(g), seed=5)
    print(f"[gpu] served mix of {len(reqs)} at full size", flush=True, file=sys.stderr)
    srv = wg.Server(0, slots=4)
    try:
        jobs = [srv.submit(r.query, to_gpu(r.src), to_gpu(r.dst)) for r in reqs]
        for i, (r, j, rec) in enumerate(zip(reqs, jobs, g)):
            s, d, st, info = j.wait()
            j.close()
            assert info["status"] == wg.WG_OK
            assert (r.query, int(r.src.size)) == (rec["query"], rec["edges"])
            assert st["result_tuples"] == rec["size"] and st["iterations"] == rec["iterations"], i
            a_s, a_d, a_st = engine.solve(r.query, to_gpu(r.src), to_gpu(r.dst))
            assert a_st["iterations"] == st["iterations"] and a_st["delta_sizes"] == st["delta_sizes"], i
            assert torch.equal(a_s, s) and torch.equal(a_d, d), i
            assert _sha(s.cpu().numpy(), d.cpu().numpy()) == rec["sha256"], i
            del s, d, a_s, a_d
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["max_running"] >= 2


def test_job_handle_outlives_server(engine):
    """Job handles freed after the server is gone (e.g. a test that failed before closing
    them) must neither touch the destroyed server nor leak the unclaimed result."""
    srv = wg.Server(0, slots=2, mem_budget_bytes=1 << 30)
    reqs = inputs.served_requests(3, seed=23, n_lo=100, n_hi=400)
    jobs = [srv.submit(r.query, to_gpu(r.src), to_gpu(r.dst)) for r in reqs]
    jobs[0].wait(want_result=False)
    srv.close()
    for j in jobs:
        assert j.done()
        j.cancel()
        info = j.info()
        assert info["phase"] == 2
        j.close()


def test_small_request_starts_beside_the_job_after_a_large_solve(engine):
    """The long-solve hold looks at the candidate counts a running solve has read back.  A
    slot that has just finished a large solve must not pass that count on to the job it
    takes next: here a long solve that never reaches 2^21 candidates (TC on a 1,500-vertex
    chain: 1,500 small iterations) and a small request wait behind a large solve's hold;
    when it ends, its slot takes the chain and the other slot must start the small request
    at once, which therefore ends first (instead of waiting for the chain)."""
    w = inputs.workload("tc_rmat_s15")
    big = (to_gpu(w.src), to_gpu(w.dst))
    chain = [to_gpu(x) for x in inputs.chain(1500)]
    tiny = inputs.erdos_renyi(300, 280, seed=1)
    tiny_gpu = [to_gpu(x) for x in tiny]
    srv = wg.Server(0, slots=2)  # the default 8 ms / 2^21-candidate hold
    try:
        srv.submit("tc", *big).wait(want_result=False)  # (warm-up)
        print("[gpu] serve: chain and small request behind a large solve", flush=True, file=sys.stderr)
        jl = srv.submit("tc", *big)
        time.sleep(0.003)  # past its first host check: a large iteration holds admissions
        jx = srv.submit("tc", *chain)
        jy = srv.submit("tc", *tiny_gpu)
        ys, yd, _, yi = jy.wait()
        _, _, xst, xi = jx.wait(want_result=False)
        _, _, lst, li = jl.wait(want_result=False)
        for j in (jl, jx, jy):
            j.close()
    finally:
        srv.close()
    assert max(lst["delta_sizes"]) >= 1 << 21
    assert xst["result_tuples"] == 1500 * 1499 // 2
    ref = oracle.tc(*tiny)
    np.testing.assert_array_equal(ys.cpu().numpy(), ref.src)
    np.testing.assert_array_equal(yd.cpu().numpy(), ref.dst)
    assert yi["end_ms"] < xi["end_ms"], (li, xi, yi)
