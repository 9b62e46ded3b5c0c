"""Device-side construction of the large Chung-Lu workload with PyTorch tensor ops.

Draws exactly the same graph as :func:`graphgen.chung_lu` (same counter-based splitmix64 streams,
same alias tables exported from the C++ generator, same planted block), but samples the endpoint
pairs and builds the symmetric, de-duplicated CSR on the GPU, which takes seconds instead of
minutes for ~10^9 entries. Holds no k-core arithmetic.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _load, Graph

M64 = (1 << 64) - 1


def _s64(x: int) -> int:
    x &= M64
    return x - (1 << 64) if x >> 63 else x


def _splitmix_host(x: int) -> int:
    x = (x + 0x9E3779B97F4A7C15) & M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & M64
    return x ^ (x >> 31)


def stream_key(seed: int, s: int) -> int:
    return _splitmix_host((seed ^ _splitmix_host((s + 0x632BE59BD9B4E019) & M64)) & M64)


_C1, _C2, _C3 = _s64(0x9E3779B97F4A7C15), _s64(0xBF58476D1CE4E5B9), _s64(0x94D049BB133111EB)


def _srl(x, k):
    # logical right shift of int64 bit patterns
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix(x):
    """splitmix64 on an int64 tensor holding uint64 bit patterns (wrapping arithmetic)."""
    x = x + _C1
    x = (x ^ _srl(x, 30)) * _C2
    x = (x ^ _srl(x, 27)) * _C3
    return x ^ _srl(x, 31)


def u01(r):
    import torch
    return _srl(r, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def chung_lu_tables(n, gamma, pairs, max_deg, block_n, block_p, seed):
    lib = _load()
    lib.gg_chung_lu_tables.restype = ctypes.c_void_p
    lib.gg_chung_lu_tables.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_double, ctypes.c_uint64]
    lib.gg_cl_block_pairs.restype = ctypes.c_int64
    lib.gg_cl_block_pairs.argtypes = [ctypes.c_void_p]
    lib.gg_cl_fill.restype = None
    lib.gg_cl_fill.argtypes = [ctypes.c_void_p] * 4
    lib.gg_cl_free.restype = None
    lib.gg_cl_free.argtypes = [ctypes.c_void_p]
    h = lib.gg_chung_lu_tables(n, gamma, pairs, max_deg, block_n, block_p, seed)
    if not h:
        raise ValueError("chung_lu_tables rejected its arguments")
    try:
        nb = lib.gg_cl_block_pairs(h)
        prob = np.empty(n, dtype=np.float64)
        alias = np.empty(n, dtype=np.int32)
        bp = np.empty(2 * nb, dtype=np.int32)
        lib.gg_cl_fill(h, prob.ctypes.data, alias.ctypes.data, bp.ctypes.data)
    finally:
        lib.gg_cl_free(h)
    return prob, alias, bp.reshape(-1, 2)


def chung_lu_device(n, gamma, pairs, max_deg, block_n, block_p, seed, device="cuda",
                    chunk=1 << 26):
    """(offsets int64[n+1], adj int32[m]) on ``device``; identical to graphgen.chung_lu."""
    import torch
    prob_h, alias_h, bp = chung_lu_tables(n, gamma, pairs, max_deg, block_n, block_p, seed)
    prob = torch.from_numpy(prob_h).to(device)
    alias = torch.from_numpy(alias_h).to(device).to(torch.int64)
    k23 = _s64(stream_key(seed, 23))
    k24 = _s64(stream_key(seed, 24))

    def draw(j):
        r1 = splitmix(j + k23)
        r2 = splitmix(j + k24)
        i = torch.clamp((u01(r1) * float(n)).to(torch.int64), max=n - 1)
        return torch.where(u01(r2) < prob[i], i, alias[i])

    keys = []
    for c0 in range(0, pairs, chunk):
        c1 = min(pairs, c0 + chunk)
        j = torch.arange(c0, c1, dtype=torch.int64, device=device) * 2
        s = draw(j)
        d = draw(j + 1)
        del j
        keep = s != d
        s, d = s[keep], d[keep]
        keys.append(s * n + d)
        keys.append(d * n + s)
        del s, d, keep
    if len(bp):
        b = torch.from_numpy(bp.astype(np.int64)).to(device)
        keys.append(b[:, 0] * n + b[:, 1])
        keys.append(b[:, 1] * n + b[:, 0])
        del b
    allk = torch.cat(keys)
    del keys
    uk = torch.unique(allk, sorted=True)
    del allk
    src = uk // n
    adj = (uk - src * n).to(torch.int32)
    del uk
    # keys are sorted, so row starts are where the source id first reaches each vertex
    offsets = torch.searchsorted(src, torch.arange(n + 1, dtype=torch.int64, device=device))
    del src
    return offsets, adj


def config_chung_lu_device(n=1 << 24, block_n=5000, device="cuda"):
    """The 16M-vertex Chung-Lu workload (see graphgen.config_chung_lu), built on the device."""
    return chung_lu_device(n, 2.1, 32 * n, 1_000_000, block_n, 0.8, 3, device=device)


def to_host(offsets, adj, name="") -> Graph:
    return Graph(offsets.cpu().numpy(), adj.cpu().numpy(), None, name)


def hcns_device(K: int, device="cuda", rows_per_chunk: int = 512):
    """Staircase graph with coreness K (the shape of the paper's HCNS): a clique on vertices
    0..K plus vertices u_i = K + i (1 <= i < K) adjacent to clique vertices 0..i-1, built on the
    device as a CSR with sorted rows. n = 2K, 2K^2 directed entries; by construction u_i has
    coreness i and the clique K (the same graph as the small test generator)."""
    import torch
    n = 2 * K
    c = torch.arange(K + 1, dtype=torch.int64, device=device)
    deg = torch.empty(n, dtype=torch.int64, device=device)
    deg[:K + 1] = K + torch.clamp(K - 1 - c, min=0)
    deg[K + 1:] = torch.arange(1, K, dtype=torch.int64, device=device)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(deg, 0)
    m = int(offsets[-1])
    adj = torch.empty(m, dtype=torch.int32, device=device)
    t = torch.arange(2 * K, dtype=torch.int64, device=device)
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=device)[:, None]
        d = deg[r0:r1][:, None]
        w = int(deg[r0:r1].max())
        tt = t[None, :w]
        clique_row = rows <= K
        # clique row c: 0..K without c, then K + c + 1, K + c + 2, ...; staircase row K + i: 0..i-1
        v_clique = torch.where(tt < rows, tt, torch.where(tt < K, tt + 1, tt + 1 + rows))
        v = torch.where(clique_row, v_clique, tt)
        mask = tt < d
        adj[int(offsets[r0]):int(offsets[r1])] = v[mask].to(torch.int32)
    return offsets, adj
