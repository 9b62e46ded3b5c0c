"""Hand-built test graphs with known coreness, and a pure-Python definition check.

Everything here is test-side only. Each family comes with the coreness that the mathematics
fixes (closed forms), so it pins the oracle independently of how the oracle computes.
"""
from __future__ import annotations

import itertools

import numpy as np

import graphgen as gg


def csr(n, edges):
    g = gg.from_edges(n, list(edges))
    return g.offsets, g.adj


def complete(n):
    return csr(n, itertools.combinations(range(n), 2))


def cycle(n):
    return csr(n, [(i, (i + 1) % n) for i in range(n)])


def path(n):
    return csr(n, [(i, i + 1) for i in range(n - 1)])


def star(leaves):
    return csr(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def random_tree(n, rng):
    return csr(n, [(i, int(rng.integers(0, i))) for i in range(1, n)])


def grid(s):
    """Plain s x s 4-neighbour grid, id = i*s + j."""
    e = []
    for i in range(s):
        for j in range(s):
            if j + 1 < s:
                e.append((i * s + j, i * s + j + 1))
            if i + 1 < s:
                e.append((i * s + j, (i + 1) * s + j))
    return csr(s * s, e)


def cube(s):
    """Plain s x s x s 6-neighbour lattice."""
    def vid(i, j, k):
        return (i * s + j) * s + k
    e = []
    for i in range(s):
        for j in range(s):
            for k in range(s):
                if i + 1 < s:
                    e.append((vid(i, j, k), vid(i + 1, j, k)))
                if j + 1 < s:
                    e.append((vid(i, j, k), vid(i, j + 1, k)))
                if k + 1 < s:
                    e.append((vid(i, j, k), vid(i, j, k + 1)))
    return csr(s ** 3, e)


def complete_bipartite(a, b):
    return csr(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def hypercube(d):
    n = 1 << d
    return csr(n, [(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)])


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return csr(10, outer + spokes + inner)


def hcns(K):
    """Staircase graph with coreness K: a clique on K+1 vertices (ids 0..K) plus vertices
    u_i (id K+i, 1 <= i < K) adjacent to clique vertices 0..i-1; coreness(u_i) = i and the clique
    has coreness K. n = 2K, directed entries = 2K^2."""
    e = list(itertools.combinations(range(K + 1), 2))
    for i in range(1, K):
        e += [(K + i, c) for c in range(i)]
    return csr(2 * K, e)


def hcns_expected(K):
    return np.array([K] * (K + 1) + list(range(1, K)), dtype=np.int32)


def union(parts):
    """Disjoint union of CSR graphs (ids shifted)."""
    offs, adjs, base, ebase = [np.zeros(1, np.int64)], [], 0, 0
    for off, adj in parts:
        n = off.shape[0] - 1
        offs.append(off[1:] + ebase)
        adjs.append(adj + np.int32(base))
        base += n
        ebase += int(off[-1])
    return np.concatenate(offs), (np.concatenate(adjs) if adjs else np.zeros(0, np.int32))


def all_graphs(n):
    """Every labelled simple graph on n vertices, as one disjoint union (graph index-major)."""
    pairs = list(itertools.combinations(range(n), 2))
    parts = []
    for mask in range(1 << len(pairs)):
        parts.append(csr(n, [p for b, p in enumerate(pairs) if mask >> b & 1]))
    return parts


def brute_py(off, adj):
    """The definition, in pure Python: v is in G_k iff it survives repeated deletion of vertices
    with fewer than k live neighbours; coreness = the largest such k."""
    n = len(off) - 1
    nb = [adj[off[v]:off[v + 1]].tolist() for v in range(n)]
    core = [0] * n
    k = 1
    while True:
        alive = [True] * n
        changed = True
        while changed:
            changed = False
            for v in range(n):
                if alive[v] and sum(alive[u] for u in nb[v]) < k:
                    alive[v] = False
                    changed = True
        if not any(alive):
            return np.array(core, dtype=np.int32)
        for v in range(n):
            if alive[v]:
                core[v] = k
        k += 1


def core_certificate(off, adj, core, stamp=None):
    """Checks, in O(m), that ``core`` is the coreness.

    (a) every v has at least core[v] neighbours u with core[u] >= core[v], so {core >= k} has
        minimum degree >= k and lies inside the k-core;
    (b) with ``stamp`` (the subround that peeled each vertex), ordering vertices by
        (core, stamp) leaves every v with at most core[v] neighbours at or after its own position,
        so v cannot belong to the (core[v]+1)-core.
    (a) and (b) together fix the coreness exactly. Returns a list of failure strings."""
    off = np.asarray(off)
    adj = np.asarray(adj)
    core = np.asarray(core, dtype=np.int64)
    n = len(off) - 1
    deg = np.diff(off)
    src = np.repeat(np.arange(n), deg)
    bad = []
    ge = np.bincount(src, weights=(core[adj] >= core[src]), minlength=n)
    if np.any(ge < core):
        bad.append(f"(a) fails at {int(np.argmax(ge < core))}")
    if stamp is not None:
        key = core * (1 << 32) + np.asarray(stamp, dtype=np.int64)
        later = np.bincount(src, weights=(key[adj] >= key[src]), minlength=n)
        if np.any(later > core):
            bad.append(f"(b) fails at {int(np.argmax(later > core))}")
    return bad
