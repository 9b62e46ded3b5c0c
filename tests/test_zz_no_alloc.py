"""The no-allocation batched entry point (kcore_decompose_batched_noalloc) against the ordinary
batched entry point and the oracle, element by element, on two calls in a row whose second input
is smaller (the scratch array keeps the first call's contents). Called through the C ABI."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import say, to_dev, first_mismatch

pytestmark = pytest.mark.gpu


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _run_both(b):
    import torch
    import paper_2502_08042_amd as K
    lib = K.lib()
    G = len(b.vptr) - 1
    d_off, d_adj, d_vptr = to_dev(b.offsets, b.adj, b.vptr)
    want_out = torch.full((b.n,), -7, dtype=torch.int32, device="cuda")
    got_out = torch.full((b.n,), -7, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = lib.kcore_decompose_batched(d_vptr.data_ptr(), d_off.data_ptr(), d_adj.data_ptr(), G, b.n,
                                     want_out.data_ptr(), _stream())
    assert rc == 0, K.last_error()
    rc = lib.kcore_decompose_batched_noalloc(d_vptr.data_ptr(), d_off.data_ptr(), d_adj.data_ptr(), G, b.n,
                                             got_out.data_ptr(), status.data_ptr(), _stream())
    assert rc == 0, K.last_error()
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 0
    return got_out.cpu().numpy(), want_out.cpu().numpy()


def test_no_alloc_batched_matches_the_allocating_entry_point_twice():
    # first call: graphs beyond the LDS capacity too (their state lives in the scratch array);
    # second call: a smaller batch on the same scratch, which still holds the first call's state
    first = gg.batch(160, 4, hi=60000)
    second = gg.batch(40, 9, hi=12000)
    assert second.n < first.n and len(second.vptr) < len(first.vptr)
    for name, b in (("first", first), ("second", second)):
        say(f"[gpu] no-alloc batched {name}: G={len(b.vptr) - 1} V={b.n} m={b.m}")
        got, want_lib = _run_both(b)
        want = oracle.bz(b.offsets, b.adj)
        assert not first_mismatch(want_lib, want), first_mismatch(want_lib, want)
        assert not first_mismatch(got, want_lib), first_mismatch(got, want_lib)


def test_no_alloc_rejects_sizes_beyond_its_scratch():
    import paper_2502_08042_amd as K
    lib = K.lib()
    say("[gpu] no-alloc size limits (host-side rejection)")
    rc = lib.kcore_decompose_batched_noalloc(None, None, None, 1, (1 << 20) + 1, None, None, _stream())
    assert rc == K.ERRORS_BY_NAME["ETOOBIG"] and "at most" in K.last_error()
    rc = lib.kcore_decompose_batched_noalloc(None, None, None, (1 << 16) + 1, 10, None, None, _stream())
    assert rc == K.ERRORS_BY_NAME["ETOOBIG"]
    assert lib.kcore_decompose_batched_noalloc(None, None, None, 0, 0, None, None, _stream()) == 0
