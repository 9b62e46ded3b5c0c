"""The racy default path, repeated, and the checked build.

Chained mode lets scans and chains of one round race for the same vertices, with the peeled bit
as the arbiter, and applies every decrement with an atomic: the online peel of Alg. 3, whose
argument is that the decrement taking a vertex to k happens exactly once. Repeating the
decomposition many times in one process must give the oracle's coreness every time. The checked
build of the library (same C ABI, kernels compiled with run-time invariant checks) must report
no violation: each coreness written exactly once, no induced degree below zero.
"""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
import graphs as G
from gpu_util import say, to_dev, run_single, first_mismatch

pytestmark = pytest.mark.gpu


def _cases():
    g = gg.grid_road(1024, 0.05, 0.01, 2)
    yield "road1024", g.offsets, g.adj
    g = gg.config_rmat16()
    yield "rmat16", g.offsets, g.adj
    off, adj = G.hcns(200)
    yield "hcns200", off, adj


def test_chained_mode_repeated_twenty_times():
    for name, off, adj in _cases():
        want = oracle.bz(off, adj)
        for rep in range(20):
            say(f"[gpu] repeat chained {name} #{rep}")
            got, st = run_single(off, adj, mode="chained")
            assert not first_mismatch(got, want), f"{name} run {rep}: {first_mismatch(got, want)}"
            assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj), (name, rep, st)
            assert st["device_status"] == 0, (name, rep, st)


def _checked_single(off, adj, mode, **tuning):
    import torch
    import paper_2502_08042_amd as K
    lib = K.lib_checked()
    d_off, d_adj = to_dev(off, adj)
    n = len(off) - 1
    out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    o = K._options(mode, False, len(adj), **tuning)
    st = K.Stats()
    rc = lib.kcore_decompose_ex(d_off.data_ptr(), d_adj.data_ptr() if len(adj) else None, n,
                                out.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                ctypes.byref(o), ctypes.byref(st))
    msg = (lib.kcore_last_error() or b"").decode()
    return rc, msg, out[:n].cpu().numpy(), st.as_dict()


@pytest.mark.parametrize("mode,tuning", [("chained", {}), ("chained", {"tail": -1}),
                                         ("levelsync", {}), ("offline", {"tail": -1}),
                                         ("chained", {"hub_degree": 16, "tile_edges": 64})])
def test_checked_build_reports_no_violation(mode, tuning):
    for name, off, adj in _cases():
        want = oracle.bz(off, adj)
        reps = 5 if mode == "chained" and not tuning else 1
        for rep in range(reps):
            say(f"[gpu] checked build {name} mode={mode} {tuning} #{rep}")
            rc, msg, got, st = _checked_single(off, adj, mode, **tuning)
            assert rc == 0, (name, msg, st)
            assert st["device_status"] == 0, (name, st)
            assert not first_mismatch(got, want), f"{name}: {first_mismatch(got, want)}"


def test_checked_build_batched():
    import torch
    import paper_2502_08042_amd as K
    lib = K.lib_checked()
    b = gg.batch(96, 4, hi=60000)
    want = oracle.bz(b.offsets, b.adj)
    d_off, d_adj, d_vptr = to_dev(b.offsets, b.adj, b.vptr)
    for mode in ("levelsync", "chained"):
        out = torch.empty(b.n, dtype=torch.int32, device="cuda")
        o = K._options(mode, False, b.m)
        st = K.Stats()
        say(f"[gpu] checked build batched G=96 mode={mode}")
        rc = lib.kcore_decompose_batched_ex(d_vptr.data_ptr(), d_off.data_ptr(), d_adj.data_ptr(), 96, b.n,
                                            out.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                            ctypes.byref(o), ctypes.byref(st))
        assert rc == 0, (lib.kcore_last_error() or b"").decode()
        assert st.device_status == 0
        assert not first_mismatch(out.cpu().numpy(), want)


def test_checked_build_multi_bucket():
    for name, off, adj in _cases():
        want = oracle.bz(off, adj)
        for mode in ("chained", "levelsync"):
            say(f"[gpu] checked build buckets {name} mode={mode}")
            rc, msg, got, st = _checked_single(off, adj, mode, buckets=1 << 30, tail=-1)
            assert rc == 0, (name, msg, st)
            assert st["device_status"] == 0, (name, st)
            assert not first_mismatch(got, want), f"{name}: {first_mismatch(got, want)}"
