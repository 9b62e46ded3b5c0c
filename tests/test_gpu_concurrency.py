"""GPU test of calls from several host threads, each on a stream of its own.

Every thread decomposes the same small set of graphs (single-graph calls in both peel modes, and a
batched call) several times in a rotated order; every result must equal the oracle's. The
single-graph peel is a persistent grid that fills the device, so the library runs those grids one
after another across streams; batched and tail launches overlap freely with them.
"""
import threading

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import say, to_dev, first_mismatch

pytestmark = pytest.mark.gpu


def test_calls_from_threads_on_distinct_streams():
    import torch
    import paper_2502_08042_amd as K
    graphs = [gg.rmat(13, 8, 21), gg.rmat(12, 16, 22), gg.grid_road(120, 0.05, 0.01, 23)]
    want = [oracle.bz(g.offsets, g.adj) for g in graphs]
    dev = [to_dev(g.offsets, g.adj) for g in graphs]
    b = gg.batch(48, 24, hi=20000)
    want_b = oracle.bz(b.offsets, b.adj)
    d_boff, d_badj, d_bvptr = to_dev(b.offsets, b.adj, b.vptr)
    torch.cuda.synchronize()
    errors = []

    def worker(t):
        s = torch.cuda.Stream()
        try:
            with torch.cuda.stream(s):
                for r in range(3):
                    for j in range(len(graphs) + 1):
                        i = (j + t) % (len(graphs) + 1)
                        if i == len(graphs):
                            got = K.decompose_batched(d_bvptr, d_boff, d_badj)
                            s.synchronize()
                            bad = first_mismatch(got.cpu().numpy(), want_b)
                        else:
                            mode = "levelsync" if (r + t) % 2 else "chained"
                            got = K.decompose(*dev[i], mode=mode)
                            s.synchronize()
                            bad = first_mismatch(got.cpu().numpy(), want[i])
                        if bad:
                            errors.append(f"thread {t} pass {r} item {i}: {bad}")
        except Exception as e:  # reported below, from the main thread
            errors.append(f"thread {t}: {e!r}")

    say("[gpu] 3 threads x 3 passes over 3 graphs + 1 batch, one stream each")
    ths = [threading.Thread(target=worker, args=(t,)) for t in range(3)]
    for th in ths:
        th.start()
    for th in ths:
        th.join(timeout=90)
    assert not any(th.is_alive() for th in ths), "a worker thread did not finish"
    assert not errors, errors[:5]
