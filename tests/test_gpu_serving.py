"""GPU tests of the batched path at full size and of the serving runtime.

Serving: each request's coreness must be identical alone and in the mix (exact integers), a tiny
HBM budget must queue requests rather than fail them, cancellation and the poll protocol must
behave as documented.
"""
import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
import graphs as G
from gpu_util import say, run_batched, first_mismatch

pytestmark = pytest.mark.gpu


def test_batched_full_4096_graphs():
    b = gg.config_batch()
    say(f"[gpu] batched full config G=4096 V={b.n} m={b.m}")
    got, st = run_batched(b.offsets, b.adj, b.vptr)
    want = oracle.bz(b.offsets, b.adj)
    assert not first_mismatch(got, want), first_mismatch(got, want)
    assert st["edges"] == b.m


def _pool():
    pool = gg.batch(48, 9, hi=30000)
    graphs = [pool.subgraph(g) for g in range(48)]
    graphs += [gg.rmat(14, 16, 77), gg.grid_road(300, 0.05, 0.01, 8)]
    return graphs


def test_serving_alone_equals_in_mix():
    import paper_2502_08042_amd as K
    graphs = _pool()
    want = [oracle.bz(g.offsets, g.adj) for g in graphs]
    say(f"[gpu] serving: {len(graphs)} graphs alone")
    with K.Server(device=0, max_inflight=3) as s:
        alone = []
        for g in graphs:
            alone.append(s.wait(s.submit(g.offsets, g.adj)))
    for a, w in zip(alone, want):
        assert np.array_equal(a, w)
    say("[gpu] serving: mixed open-loop stream from two threads")
    rng = np.random.default_rng(1)
    order = rng.integers(0, len(graphs), 600)
    with K.Server(device=0, max_inflight=4, max_batch_graphs=64) as s:
        tickets = [None] * len(order)

        def producer(lo, hi):
            for i in range(lo, hi):
                g = graphs[order[i]]
                tickets[i] = s.submit(g.offsets, g.adj)
                if i % 7 == 0:
                    time.sleep(0.0005)

        ths = [threading.Thread(target=producer, args=(0, 300)),
               threading.Thread(target=producer, args=(300, 600))]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        batches = set()
        for i, t in enumerate(tickets):
            core, st = s.wait(t, with_stats=True)
            assert np.array_equal(core, want[order[i]]), f"request {i} differs from alone"
            assert st["submit_us"] <= st["admit_us"] <= st["launch_us"] <= st["done_us"]
            batches.add(st["batch_id"])
        assert len(batches) > 1


def test_serving_budget_queues_instead_of_failing():
    import paper_2502_08042_amd as K
    graphs = _pool()[:20]
    biggest = max(8 * (g.n + 1) + 4 * g.m + 16 * g.n + 64 for g in graphs)
    say("[gpu] serving: budget fits one request at a time")
    with K.Server(device=0, max_inflight=4, hbm_budget_bytes=biggest) as s:
        ts = [s.submit(g.offsets, g.adj) for g in graphs]
        for t, g in zip(ts, graphs):
            core, st = s.wait(t, with_stats=True)
            assert np.array_equal(core, oracle.bz(g.offsets, g.adj))
            assert st["batch_graphs"] >= 1
        # a request that can never fit is refused at submit time
        off, adj = G.complete(200)
        with pytest.raises(K.KcoreError) as e:
            s2 = K.Server(device=0, hbm_budget_bytes=1000)
            try:
                s2.submit(off, adj)
            finally:
                s2.close()
        assert e.value.code == -4


def test_serving_poll_protocol_and_cancel():
    import paper_2502_08042_amd as K
    off, adj = G.hcns(50)
    say("[gpu] serving: poll protocol")
    with K.Server(device=0, max_inflight=1) as s:
        t = s.submit(off, adj)
        core = s.wait(t)
        assert np.array_equal(core, G.hcns_expected(50))
        rc = K.lib().kcore_poll(s._h, t, None, None)
        assert rc == -5  # result already taken
        # an empty graph completes at once
        t0 = s.submit(np.zeros(1, np.int64), np.zeros(0, np.int32))
        assert s.wait(t0).shape == (0,)
        # cancel: flood the queue, cancel the last request before it can start
        big = gg.rmat(16, 16, 3)
        ts = [s.submit(big.offsets, big.adj) for _ in range(6)]
        rc = s.cancel(ts[-1])
        assert rc in (0, 1)
        for tt in ts[:-1]:
            s.wait(tt)
        if rc == 0:
            with pytest.raises(K.KcoreError) as e:
                s.wait(ts[-1])
            assert e.value.code == -6
        else:
            s.wait(ts[-1])


def test_serving_injected_launch_failure_fails_only_its_request():
    """A launch failure forced on one ticket (before any device work) fails that request alone: its
    batch is retried one request per batch, and every other request completes exactly."""
    import paper_2502_08042_amd as K
    graphs = _pool()[:16]
    want = [oracle.bz(g.offsets, g.adj) for g in graphs]
    say("[gpu] serving: injected launch failure on ticket 5")
    with K.Server(device=0, max_inflight=2, fail_ticket=5) as s:
        ts = [s.submit(g.offsets, g.adj) for g in graphs]
        assert ts[4] == 5
        for i, (t, w) in enumerate(zip(ts, want)):
            if t == 5:
                with pytest.raises(K.KcoreError) as e:
                    s.wait(t)
                assert e.value.code == -3
            else:
                assert np.array_equal(s.wait(t), w), f"request {i}"


def test_serving_size_classes_never_share_a_batch():
    """Small (held in LDS by the batched peel), medium (more vertices than that) and large
    (large_vertices and up) requests run in batches of their own class; results stay exact."""
    import paper_2502_08042_amd as K
    small = [gg.batch(24, 10, hi=3000).subgraph(g) for g in range(24)]
    medium = [gg.rmat(14, 8, 40 + i) for i in range(4)]       # 16,384 vertices
    large = [gg.rmat(15, 8, 50 + i) for i in range(2)]        # 32,768 vertices with large_vertices 20,000
    graphs = small[:8] + medium[:2] + small[8:16] + large[:1] + medium[2:] + small[16:] + large[1:]
    cls = {id(g): c for c, gs in (("small", small), ("medium", medium), ("large", large)) for g in gs}
    want = [oracle.bz(g.offsets, g.adj) for g in graphs]
    say(f"[gpu] serving: {len(graphs)} requests of three size classes")
    with K.Server(device=0, max_inflight=4, max_large_inflight=1, large_vertices=20000) as s:
        ts = [s.submit(g.offsets, g.adj) for g in graphs]
        by_batch = {}
        for t, g, w in zip(ts, graphs, want):
            core, st = s.wait(t, with_stats=True)
            assert np.array_equal(core, w)
            by_batch.setdefault(st["batch_id"], set()).add(cls[id(g)])
    assert all(len(c) == 1 for c in by_batch.values()), by_batch
    assert {next(iter(c)) for c in by_batch.values()} == {"small", "medium", "large"}
