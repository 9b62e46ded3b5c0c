"""Helpers for GPU tests: move host CSR to the device, run the library, compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(off, adj, vptr=None):
    import torch
    d_off = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).cuda()
    d_adj = torch.from_numpy(np.ascontiguousarray(adj, dtype=np.int32)).cuda()
    if vptr is None:
        return d_off, d_adj
    return d_off, d_adj, torch.from_numpy(np.ascontiguousarray(vptr, dtype=np.int64)).cuda()


def run_single(off, adj, mode="auto", stats=True, **kw):
    import torch
    import paper_2502_08042_amd as K
    d_off, d_adj = to_dev(off, adj)
    r = K.decompose(d_off, d_adj, mode=mode, stats=stats, **kw)
    torch.cuda.synchronize()
    if stats:
        core, st = r
        return core.cpu().numpy(), st
    return r.cpu().numpy(), None


def run_batched(off, adj, vptr, stats=True, mode="auto"):
    import torch
    import paper_2502_08042_amd as K
    d_off, d_adj, d_vptr = to_dev(off, adj, vptr)
    r = K.decompose_batched(d_vptr, d_off, d_adj, stats=stats, mode=mode)
    torch.cuda.synchronize()
    if stats:
        core, st = r
        return core.cpu().numpy(), st
    return r.cpu().numpy(), None


def first_mismatch(got, want):
    bad = np.nonzero(got != want)[0]
    if len(bad) == 0:
        return ""
    i = int(bad[0])
    return f"{len(bad)} mismatches, first at {i}: got {int(got[i])} want {int(want[i])}"
