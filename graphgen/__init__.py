"""Seeded synthetic graph generators (host side), shared by tests, the oracle checks and bench.py.

Holds no k-core arithmetic: these functions only draw graphs and return them as numpy CSR
arrays ``(offsets int64[n+1], adj int32[nnz])`` with both directions of every undirected edge,
sorted rows, no self-loops and no duplicate entries. All randomness is counter-based
(splitmix64 keyed by seed, stream, index), so outputs do not depend on the thread count.

The workload recipes (``config_*``) reproduce the shapes the benchmark and the parity tests use:
R-MAT scale 16, a road-like 4096^2 grid, a 16M-vertex Chung-Lu power law with a planted dense
block, a 4096-graph segmented batch and a serving request pool.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the generator library with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, u64, f64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32
    lib.gg_rmat.restype = P
    lib.gg_rmat.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64]
    lib.gg_rmat_n.restype = P
    lib.gg_rmat_n.argtypes = [i64, i64, f64, f64, f64, u64]
    lib.gg_grid_road.restype = P
    lib.gg_grid_road.argtypes = [i64, f64, f64, u64]
    lib.gg_chung_lu.restype = P
    lib.gg_chung_lu.argtypes = [i64, f64, i64, i64, i64, f64, u64]
    lib.gg_erdos_renyi.restype = P
    lib.gg_erdos_renyi.argtypes = [i64, f64, u64]
    lib.gg_from_edges.restype = P
    lib.gg_from_edges.argtypes = [i64, i64, P, P]
    lib.gg_batch.restype = P
    lib.gg_batch.argtypes = [i32, i64, u64, f64, f64, i64, i64, f64, i64, f64, f64, f64]
    for f in ("gg_num_vertices", "gg_num_entries", "gg_num_graphs"):
        getattr(lib, f).restype = i64
        getattr(lib, f).argtypes = [P]
    lib.gg_fill.restype = ctypes.c_int
    lib.gg_fill.argtypes = [P, P, P, P]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [P]
    lib.gg_uniform.restype = None
    lib.gg_uniform.argtypes = [u64, u64, u64, i64, P]
    _lib = lib
    return lib


@dataclass
class Graph:
    """Host CSR. ``vptr`` (int64[G+1]) is set for segmented batches of independent graphs."""
    offsets: np.ndarray
    adj: np.ndarray
    vptr: np.ndarray | None = None
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        """Directed CSR entries (both directions of each undirected edge)."""
        return int(self.adj.shape[0])

    def subgraph(self, g: int) -> "Graph":
        """Graph ``g`` of a segmented batch, renumbered from 0."""
        assert self.vptr is not None
        lo, hi = int(self.vptr[g]), int(self.vptr[g + 1])
        e0, e1 = int(self.offsets[lo]), int(self.offsets[hi])
        return Graph(self.offsets[lo:hi + 1] - e0, self.adj[e0:e1] - np.int32(lo), None,
                     f"{self.name}[{g}]")


def _take(h, name: str) -> Graph:
    lib = _load()
    if not h:
        raise ValueError(f"graph generator rejected its arguments ({name})")
    try:
        n = lib.gg_num_vertices(h)
        nnz = lib.gg_num_entries(h)
        G = lib.gg_num_graphs(h)
        off = np.empty(n + 1, dtype=np.int64)
        adj = np.empty(nnz, dtype=np.int32)
        vptr = np.empty(G + 1, dtype=np.int64) if G > 0 else None
        lib.gg_fill(h, off.ctypes.data, adj.ctypes.data, vptr.ctypes.data if vptr is not None else None)
    finally:
        lib.gg_free(h)
    return Graph(off, adj, vptr, name)


RMAT_ABC = (0.57, 0.19, 0.19)


def rmat(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC) -> Graph:
    return _take(_load().gg_rmat(scale, edge_factor, *abc, seed), f"rmat{scale}x{edge_factor}")


def rmat_n(n: int, draws: int, seed: int, abc=RMAT_ABC) -> Graph:
    return _take(_load().gg_rmat_n(n, draws, *abc, seed), f"rmat_n{n}")


def grid_road(s: int, p_del: float, p_diag: float, seed: int) -> Graph:
    return _take(_load().gg_grid_road(s, p_del, p_diag, seed), f"grid{s}")


def chung_lu(n: int, gamma: float, pairs: int, max_deg: int, block_n: int, block_p: float,
             seed: int) -> Graph:
    return _take(_load().gg_chung_lu(n, gamma, pairs, max_deg, block_n, block_p, seed),
                 f"chunglu{n}")


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    return _take(_load().gg_erdos_renyi(n, p, seed), f"er{n}")


def from_edges(n: int, edges) -> Graph:
    """Undirected edge list (pairs) -> symmetric CSR; loops dropped, duplicates merged."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint out of range")
    src = np.ascontiguousarray(e[:, 0], dtype=np.int32)
    dst = np.ascontiguousarray(e[:, 1], dtype=np.int32)
    return _take(_load().gg_from_edges(n, len(src), src.ctypes.data, dst.ctypes.data), "edges")


def batch(num_graphs: int, seed: int, first_graph: int = 0, median: float = 2000.0,
          sigma: float = 1.0, lo: int = 100, hi: int = 100_000, avg_deg: float = 8.0,
          rmat_factor: int = 8, abc=RMAT_ABC) -> Graph:
    """Segmented batch: graph g (global index first_graph+g) is the same in every batch."""
    return _take(_load().gg_batch(num_graphs, first_graph, seed, median, sigma, lo, hi, avg_deg,
                                  rmat_factor, *abc), f"batch{num_graphs}")


def uniform(seed: int, stream: int, first: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().gg_uniform(seed, stream, first, count, out.ctypes.data)
    return out


# ---- the benchmark workloads -------------------------------------------------------------

def config_rmat16() -> Graph:
    """R-MAT scale 16, edge factor 16, a=.57 b=.19 c=.19, symmetrised, seed 1."""
    g = rmat(16, 16, 1)
    g.name = "rmat16"
    return g


def config_grid4096(s: int = 4096) -> Graph:
    """Road-like grid s x s: 5% of lattice edges deleted, 1% of unit squares get a diagonal, seed 2."""
    g = grid_road(s, 0.05, 0.01, 2)
    g.name = f"grid{s}"
    return g


def config_chung_lu(n: int = 1 << 24, block_n: int = 5000) -> Graph:
    """Chung-Lu gamma=2.1, 32n endpoint pairs (~1B directed entries at n=2^24), degree cap 1e6,
    planted G(block_n, 0.8) block, seed 3."""
    g = chung_lu(n, 2.1, 32 * n, 1_000_000, block_n, 0.8, 3)
    g.name = f"chunglu{n}"
    return g


def config_batch(num_graphs: int = 4096, first_graph: int = 0) -> Graph:
    """Segmented batch of lognormal-sized ER (avg deg 8) / R-MAT (8n draws) graphs, seed 4."""
    g = batch(num_graphs, 4, first_graph=first_graph)
    g.name = f"batch{num_graphs}"
    return g


def serving_large(seed: int = 5) -> Graph:
    """The 1% serving class: R-MAT scale 20, edge factor 16."""
    g = rmat(20, 16, seed)
    g.name = "rmat20"
    return g
