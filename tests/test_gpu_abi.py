"""The C ABI on the GPU, called through ctypes exactly as a C caller would: the plain entry points
(no options: the workspace is sized without reading offsets[n] on the host), the device status
word (kcore_check, status_out) and a failure forced from the host, which must be reported.

Every case prints its name before touching the GPU."""
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


@pytest.mark.parametrize("which", ["rmat16", "road128", "road1024"])
def test_plain_decompose_through_the_c_abi(which):
    import torch
    import paper_2502_08042_amd as K
    g = gg.config_rmat16() if which == "rmat16" else gg.grid_road(int(which[4:]), 0.05, 0.01, 2)
    want = oracle.bz(g.offsets, g.adj)
    d_off, d_adj = to_dev(g.offsets, g.adj)
    out = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
    lib = K.lib()
    for rep in range(2):
        say(f"[gpu] plain kcore_decompose {which} n={g.n} m={g.m} call {rep}")
        rc = lib.kcore_decompose(d_off.data_ptr(), d_adj.data_ptr(), g.n, out.data_ptr(), _stream())
        assert rc == 0, K.last_error()
        assert lib.kcore_check(_stream()) == 0, K.last_error()
        got = out.cpu().numpy()
        assert not first_mismatch(got, want), first_mismatch(got, want)
        out.fill_(-1)


def test_plain_decompose_on_a_slice_of_a_larger_allocation():
    """adj is a view into the middle of a bigger device allocation (as when many graphs share one
    buffer): the workspace is sized from what is left of that allocation, and the result is exact."""
    import torch
    import paper_2502_08042_amd as K
    g = gg.rmat(12, 16, 11)
    want = oracle.bz(g.offsets, g.adj)
    big = torch.zeros(g.m + 5_000_000, dtype=torch.int32, device="cuda")
    lo = 1_234_567
    big[lo:lo + g.m] = torch.from_numpy(g.adj).cuda()
    d_off = torch.from_numpy(g.offsets).cuda()
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    say(f"[gpu] plain kcore_decompose on a slice at {lo}")
    rc = K.lib().kcore_decompose(d_off.data_ptr(), big[lo:].data_ptr(), g.n, out.data_ptr(), _stream())
    assert rc == 0, K.last_error()
    assert K.lib().kcore_check(_stream()) == 0, K.last_error()
    assert not first_mismatch(out.cpu().numpy(), want)


def test_plain_batched_through_the_c_abi():
    import torch
    import paper_2502_08042_amd as K
    b = gg.batch(64, 4, hi=20000)
    want = oracle.bz(b.offsets, b.adj)
    d_off, d_adj, d_vptr = to_dev(b.offsets, b.adj, b.vptr)
    out = torch.full((b.n,), -1, dtype=torch.int32, device="cuda")
    say(f"[gpu] plain kcore_decompose_batched G=64 V={b.n}")
    rc = K.lib().kcore_decompose_batched(d_vptr.data_ptr(), d_off.data_ptr(), d_adj.data_ptr(), 64,
                                         b.n, out.data_ptr(), _stream())
    assert rc == 0, K.last_error()
    assert K.lib().kcore_check(_stream()) == 0, K.last_error()
    assert not first_mismatch(out.cpu().numpy(), want)


def test_status_out_and_a_failure_forced_from_the_host():
    """num_entries below offsets[n] sizes the workspace too small: the kernel must notice before it
    reads any entry, stop, and report it through status_out and kcore_check (the call itself has
    already returned OK). The next call on the stream succeeds again."""
    import torch
    import paper_2502_08042_amd as K
    g = gg.rmat(12, 16, 11)
    want = oracle.bz(g.offsets, g.adj)
    d_off, d_adj = to_dev(g.offsets, g.adj)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32).pin_memory()
    lib = K.lib()
    for mode in ("chained", "levelsync"):
        o = K._options(mode, False, g.m // 2, status_out=status.data_ptr())
        say(f"[gpu] forced overflow mode={mode} num_entries={g.m // 2} < m={g.m}")
        rc = lib.kcore_decompose_ex(d_off.data_ptr(), d_adj.data_ptr(), g.n, out.data_ptr(), _stream(),
                                    ctypes.byref(o), None)
        assert rc == 0, K.last_error()
        assert lib.kcore_check(_stream()) == K.ERRORS_BY_NAME["EDEVICE"], K.last_error()
        assert "failure bits" in K.last_error()
        assert int(status[0]) != 0
        o = K._options(mode, False, g.m, status_out=status.data_ptr())
        say(f"[gpu] same graph with the right num_entries, mode={mode}")
        rc = lib.kcore_decompose_ex(d_off.data_ptr(), d_adj.data_ptr(), g.n, out.data_ptr(), _stream(),
                                    ctypes.byref(o), None)
        assert rc == 0, K.last_error()
        assert lib.kcore_check(_stream()) == 0, K.last_error()
        torch.cuda.synchronize()
        assert int(status[0]) == 0
        assert not first_mismatch(out.cpu().numpy(), want)


def test_check_without_any_call_on_the_stream():
    import torch
    import paper_2502_08042_amd as K
    s = torch.cuda.Stream()
    say("[gpu] kcore_check on a fresh stream")
    assert K.lib().kcore_check(ctypes.c_void_p(s.cuda_stream)) == K.ERRORS_BY_NAME["ENOTFOUND"]
