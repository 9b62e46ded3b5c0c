"""CPU oracle for exact k-core decomposition — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg may import
this package. The GPU library never calls it; the two share no code.

Functions (all take a host CSR ``offsets int64[n+1], adj int32[nnz]`` of a simple undirected graph
with both edge directions stored, and return ``int32[n]`` coreness):

* :func:`bz` — Batagelj–Zaversnik bucket peel, the sequential O(n+m) baseline of the paper
  (Sec. 1; Sec. 6.1 "Baselines"). The primary oracle.
* :func:`brute` — the k-core definition applied directly (Sec. 1, Sec. 2 "Notations").
* :func:`hindex` — h-index iteration to its fixed point (Lu et al. 2016), independent of the paper.
* :func:`levelsync` — Alg. 1 with its sequential peel, subround by subround; also returns the
  structural counts (rho, rounds, Thm. 3.1 active-set total) and each vertex's peel subround.

Parity unpinned: none — every function is pinned by tests/test_oracle.py (brute force on all
small graphs, closed forms, the h-index fixed point and Thm. 3.1 identities).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

LEVELSYNC_FIELDS = ("rounds", "nonempty_rounds", "subrounds", "frontier_total",
                    "active_total", "edges_expanded", "max_subrounds_in_round")


def build(force: bool = True, src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (plain C, -O2). ``src``/``out``/``extra`` let tests compile a
    deliberately broken copy to check that the pins catch it."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *extra, "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _bind(path: str):
    lib = ctypes.CDLL(path)
    P, i64 = ctypes.c_void_p, ctypes.c_int64
    for f in ("oracle_bz", "oracle_brute"):
        getattr(lib, f).restype = ctypes.c_int
        getattr(lib, f).argtypes = [i64, P, P, P]
    lib.oracle_hindex.restype = ctypes.c_int
    lib.oracle_hindex.argtypes = [i64, P, P, P, P]
    lib.oracle_levelsync.restype = ctypes.c_int
    lib.oracle_levelsync.argtypes = [i64, P, P, P, P, P]
    return lib


def load(path: str | None = None):
    """The compiled oracle library (built on first use)."""
    global _lib
    if path is not None:
        return _bind(path)
    if _lib is None:
        build(force=not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
        _lib = _bind(_LIB)
    return _lib


def _prep(offsets, adj):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    a = np.ascontiguousarray(adj, dtype=np.int32)
    n = off.shape[0] - 1
    if n < 0:
        raise ValueError("offsets must have n+1 entries")
    return off, a, n


def _check(rc: int, name: str):
    if rc != 0:
        raise RuntimeError(f"{name} failed with code {rc}")


def bz(offsets, adj, lib=None) -> np.ndarray:
    off, a, n = _prep(offsets, adj)
    core = np.empty(n, dtype=np.int32)
    _check((lib or load()).oracle_bz(n, off.ctypes.data, a.ctypes.data, core.ctypes.data), "oracle_bz")
    return core


def brute(offsets, adj, lib=None) -> np.ndarray:
    off, a, n = _prep(offsets, adj)
    core = np.empty(n, dtype=np.int32)
    _check((lib or load()).oracle_brute(n, off.ctypes.data, a.ctypes.data, core.ctypes.data),
           "oracle_brute")
    return core


def hindex(offsets, adj, lib=None):
    """Returns (coreness, sweeps)."""
    off, a, n = _prep(offsets, adj)
    core = np.empty(n, dtype=np.int32)
    it = ctypes.c_int64(0)
    _check((lib or load()).oracle_hindex(n, off.ctypes.data, a.ctypes.data, core.ctypes.data,
                                         ctypes.byref(it)), "oracle_hindex")
    return core, int(it.value)


def levelsync(offsets, adj, lib=None):
    """Returns (coreness, per-vertex peel subround, dict of counts named LEVELSYNC_FIELDS)."""
    off, a, n = _prep(offsets, adj)
    core = np.empty(n, dtype=np.int32)
    sub = np.empty(n, dtype=np.int32)
    st = np.zeros(7, dtype=np.int64)
    _check((lib or load()).oracle_levelsync(n, off.ctypes.data, a.ctypes.data, core.ctypes.data,
                                            sub.ctypes.data, st.ctypes.data), "oracle_levelsync")
    return core, sub, dict(zip(LEVELSYNC_FIELDS, (int(x) for x in st)))


def time_bz(offsets, adj, repeats: int = 1, core_out=None) -> list[float]:
    """Wall-clock seconds of each of ``repeats`` oracle_bz runs on one host thread; the coreness
    of the runs lands in ``core_out`` (an int32 array of n entries) when one is given."""
    off, a, n = _prep(offsets, adj)
    core = np.empty(n, dtype=np.int32) if core_out is None else core_out
    if core.dtype != np.int32 or core.shape != (n,) or not core.flags.c_contiguous:
        raise ValueError("core_out must be a contiguous int32 array of n entries")
    lib = load()
    out = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        _check(lib.oracle_bz(n, off.ctypes.data, a.ctypes.data, core.ctypes.data), "oracle_bz")
        out.append(time.perf_counter() - t0)
    return out
