"""Exact k-core decomposition on AMD Instinct MI355X — Python binding of ``libkcore.so``.

Thin ctypes marshalling over the C ABI declared in ``include/kcore.h``: every step of the
computation runs in the library's HIP kernels. PyTorch is used only to hold device memory and to
name the current HIP stream. If the library has not been built the import fails loudly; there is
no fallback.

Single graph::

    core = decompose(offsets_dev_int64, adj_dev_int32)               # int32 tensor on the device
    core, st = decompose(offsets, adj, stats=True, mode="levelsync")  # + counters dict

Batch of independent graphs in one segmented CSR (global ids)::

    core = decompose_batched(vptr_dev_int64, offsets, adj)

Serving (host graphs in, host results out)::

    with Server(device=0) as s:
        t = s.submit(offsets_np, adj_np)
        core = s.wait(t)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkcore.so")

KCORE_OK, KCORE_PENDING = 0, 1
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ETOOBIG", -5: "ENOTFOUND",
          -6: "ECANCELED", -7: "EBADGRAPH"}
ERRORS_BY_NAME = {v: k for k, v in ERRORS.items()}
MODES = {"auto": 0, "levelsync": 1, "chained": 2, "sampling": 3, "offline": 4}


class KcoreError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code}): {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("hub_degree", ctypes.c_int32),
                ("num_entries", ctypes.c_int64), ("local_budget", ctypes.c_int32),
                ("tile_edges", ctypes.c_int32), ("async_frontier", ctypes.c_int32),
                ("async_scan", ctypes.c_int32), ("block_tiles", ctypes.c_int32),
                ("block_queue", ctypes.c_int32), ("tile_probe", ctypes.c_int32),
                ("residual", ctypes.c_int32), ("tail", ctypes.c_int32),
                ("buckets", ctypes.c_int32), ("sample_threshold", ctypes.c_int32),
                ("sample_mu", ctypes.c_int32), ("debug_phase", ctypes.c_int32),
                ("test_tail_entries", ctypes.c_int64), ("team_size", ctypes.c_int32), ("combine_degree", ctypes.c_int32), ("big_phase", ctypes.c_int32),
                ("batch_teams", ctypes.c_int32), ("status_out", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("subrounds", ctypes.c_int64),
                ("barriers", ctypes.c_int64), ("peeled", ctypes.c_int64),
                ("edges", ctypes.c_int64), ("decrements", ctypes.c_int64),
                ("combined", ctypes.c_int64), ("scanned", ctypes.c_int64),
                ("kmax", ctypes.c_int32), ("device_status", ctypes.c_int32),
                ("ms", ctypes.c_float), ("tail_vertices", ctypes.c_int32),
                ("sampled_vertices", ctypes.c_int32), ("sample_recounts", ctypes.c_int32),
                ("sample_restarts", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1),
                ("live_decrements", ctypes.c_int64), ("bucket_inserts", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_graphs", ctypes.c_int32), ("max_large_inflight", ctypes.c_int32),
                ("max_batch_vertices", ctypes.c_int64), ("hbm_budget_bytes", ctypes.c_int64),
                ("max_request_vertices", ctypes.c_int64), ("batch_wait_us", ctypes.c_double),
                ("borrow_inputs", ctypes.c_int32), ("large_vertices", ctypes.c_int32),
                ("reserve_vertices", ctypes.c_int64), ("reserve_entries", ctypes.c_int64),
                ("fail_ticket", ctypes.c_uint64)]


class RequestStats(ctypes.Structure):
    _fields_ = [("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("launch_us", ctypes.c_double), ("done_us", ctypes.c_double),
                ("batch_id", ctypes.c_int64), ("batch_graphs", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


# Every exported symbol of include/kcore.h with its ctypes signature.
P, I32, I64, U64P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)
SIGNATURES = {
    "kcore_decompose": (ctypes.c_int, [P, P, I64, P, P]),
    "kcore_decompose_ex": (ctypes.c_int, [P, P, I64, P, P, ctypes.POINTER(Options), ctypes.POINTER(Stats)]),
    "kcore_kcore_subgraph": (ctypes.c_int, [P, P, I64, I32, P, P, ctypes.POINTER(Options),
                                            ctypes.POINTER(Stats)]),
    "kcore_decompose_batched": (ctypes.c_int, [P, P, P, I32, I64, P, P]),
    "kcore_decompose_batched_noalloc": (ctypes.c_int, [P, P, P, I32, I64, P, P, P]),
    "kcore_decompose_batched_ex": (ctypes.c_int, [P, P, P, I32, I64, P, P, ctypes.POINTER(Options),
                                                  ctypes.POINTER(Stats)]),
    "kcore_release_workspaces": (ctypes.c_int, []),
    "kcore_check": (ctypes.c_int, [P]),
    "kcore_server_create": (P, [ctypes.POINTER(ServerConfig)]),
    "kcore_submit": (ctypes.c_int, [P, P, P, I64, U64P]),
    "kcore_poll": (ctypes.c_int, [P, ctypes.c_uint64, P, ctypes.POINTER(RequestStats)]),
    "kcore_wait": (ctypes.c_int, [P, ctypes.c_uint64, P, ctypes.POINTER(RequestStats), ctypes.c_double]),
    "kcore_cancel": (ctypes.c_int, [P, ctypes.c_uint64]),
    "kcore_server_now_us": (ctypes.c_double, [P]),
    "kcore_server_destroy": (None, [P]),
    "kcore_last_error": (ctypes.c_char_p, []),
    "kcore_version": (ctypes.c_int, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first with "
                          "`python -c 'import __graft_entry__ as g; g.build()'` "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    # PyTorch ships its own copy of the HIP runtime under the same soname. Loading PyTorch first
    # makes the dynamic loader bind this library to that copy; the other order would put two HIP
    # (and HSA) runtimes in one process, and the one initialised second finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _release_at_exit():
    # Free the library's cached device workspaces, pinned blocks and events while the HIP runtime
    # (and any profiler attached to it) is still fully alive, instead of leaving them to process
    # teardown.
    try:
        import torch
        if torch.cuda.is_initialized():
            _lib.kcore_release_workspaces()
    except Exception:
        pass


import atexit  # noqa: E402

atexit.register(_release_at_exit)


def lib():
    return _lib


_lib_checked = None


def lib_checked():
    """The checked build of the same library (``libkcore_checked.so``): identical C ABI, but its
    kernels verify while they run that every coreness is written exactly once and that no induced
    degree goes below zero, reporting a violation through the device status word. For tests."""
    global _lib_checked
    if _lib_checked is None:
        path = os.path.join(_HERE, "libkcore_checked.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it first (it is built with libkcore.so)")
        h = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib_checked = h
    return _lib_checked


def last_error() -> str:
    return (_lib.kcore_last_error() or b"").decode()


def _check(rc: int, where: str):
    if rc != KCORE_OK:
        raise KcoreError(rc, where, last_error())


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _options(mode, validate, num_entries, hub_degree=0, local_budget=0, tile_edges=0,
             blocks_per_cu=0, async_frontier=0, async_scan=0, block_tiles=0,
             block_queue=0, tile_probe=0, residual=0, tail=0, buckets=0, sample_threshold=0,
             sample_mu=0, debug_phase=0, test_tail_entries=0, team_size=0, combine_degree=0, big_phase=0, batch_teams=0,
             status_out=None) -> Options:
    o = Options()
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.validate = 1 if validate else 0
    o.blocks_per_cu = blocks_per_cu
    o.hub_degree = hub_degree
    o.num_entries = num_entries
    o.local_budget = local_budget
    o.tile_edges = tile_edges
    o.async_frontier = async_frontier
    o.async_scan = async_scan
    o.block_tiles = block_tiles
    o.block_queue = block_queue
    o.tile_probe = tile_probe
    o.residual = residual
    o.tail = tail
    o.buckets = buckets
    o.sample_threshold = sample_threshold
    o.sample_mu = sample_mu
    o.debug_phase = debug_phase
    o.test_tail_entries = test_tail_entries
    o.team_size = team_size
    o.combine_degree = combine_degree
    o.big_phase = big_phase
    o.batch_teams = batch_teams
    o.status_out = status_out
    return o


def _dev_tensor(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on a GPU")
    return t


def decompose(offsets, adj, out=None, *, mode="auto", stats=False, validate=False, stream=None,
              tuned=False, **tuning):
    """Coreness of every vertex of one graph (device CSR: int64 offsets[n+1], int32 adj[m]).

    Returns the int32 coreness tensor (``out`` if given), plus a dict of counters when
    ``stats=True`` (that call synchronises the stream). ``tuned=True`` applies the autotuner's
    cached options for this device and the graph's workload class (explicit ``tuning`` keywords
    win)."""
    import torch
    _dev_tensor(offsets, torch.int64, "offsets")
    _dev_tensor(adj, torch.int32, "adj")
    if tuned:
        from . import autotune
        tuning = {**autotune.tuned_options(offsets), **tuning}
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=offsets.device)
    _dev_tensor(out, torch.int32, "out")
    if out.numel() < n:
        raise ValueError("out is too small")
    opt = _options(mode, validate, adj.numel(), **tuning)
    st = Stats() if stats else None
    rc = _lib.kcore_decompose_ex(offsets.data_ptr(), adj.data_ptr() if adj.numel() else None, n,
                                 out.data_ptr() if n else None, _stream_ptr(stream),
                                 ctypes.byref(opt), ctypes.byref(st) if st is not None else None)
    _check(rc, "kcore_decompose_ex")
    return (out, st.as_dict()) if stats else out


def kcore_subgraph(offsets, adj, k, out=None, *, mode="auto", stats=False, validate=False, stream=None,
                   **tuning):
    """Membership of the maximum k-core subgraph: int32 tensor, 1 for vertices of the k-core."""
    import torch
    _dev_tensor(offsets, torch.int64, "offsets")
    _dev_tensor(adj, torch.int32, "adj")
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=offsets.device)
    _dev_tensor(out, torch.int32, "out")
    if out.numel() < n:
        raise ValueError("out is too small")
    opt = _options(mode, validate, adj.numel(), **tuning)
    st = Stats() if stats else None
    rc = _lib.kcore_kcore_subgraph(offsets.data_ptr(), adj.data_ptr() if adj.numel() else None, n, int(k),
                                   out.data_ptr() if n else None, _stream_ptr(stream), ctypes.byref(opt),
                                   ctypes.byref(st) if st is not None else None)
    _check(rc, "kcore_kcore_subgraph")
    return (out, st.as_dict()) if stats else out


def decompose_batched(vptr, offsets, adj, out=None, *, mode="auto", stats=False, validate=False,
                      stream=None, tuned=False, blocks_per_cu=0, batch_teams=0, team_size=0):
    """Coreness for a segmented batch of independent graphs (device tensors, global ids).
    ``mode``: "auto"/"levelsync" (barrier-separated subrounds inside each graph's workgroup) or
    "chained" (each round peeled through a dynamic workgroup queue). ``tuned=True`` applies the
    autotuner's cached mode and workgroups per CU for this device and batch size."""
    import torch
    if tuned:
        from . import autotune
        t = autotune.tuned_options(offsets, batched=True)
        mode = t.get("mode", mode)
        blocks_per_cu = t.get("blocks_per_cu", blocks_per_cu)
        batch_teams = t.get("batch_teams", batch_teams)
        team_size = t.get("team_size", team_size)
    _dev_tensor(vptr, torch.int64, "vptr")
    _dev_tensor(offsets, torch.int64, "offsets")
    _dev_tensor(adj, torch.int32, "adj")
    G = vptr.numel() - 1
    V = offsets.numel() - 1
    if adj.numel() == 0:
        adj = torch.zeros(1, dtype=torch.int32, device=offsets.device)
    if out is None:
        out = torch.empty(max(V, 0), dtype=torch.int32, device=offsets.device)
    _dev_tensor(out, torch.int32, "out")
    opt = _options(mode, validate, adj.numel(), blocks_per_cu=blocks_per_cu, batch_teams=batch_teams,
                   team_size=team_size)
    st = Stats() if stats else None
    rc = _lib.kcore_decompose_batched_ex(vptr.data_ptr(), offsets.data_ptr(), adj.data_ptr(), G, V,
                                         out.data_ptr() if V else None, _stream_ptr(stream),
                                         ctypes.byref(opt),
                                         ctypes.byref(st) if st is not None else None)
    _check(rc, "kcore_decompose_batched_ex")
    return (out, st.as_dict()) if stats else out


def release_workspaces():
    _check(_lib.kcore_release_workspaces(), "kcore_release_workspaces")


def check(stream=None):
    """Waits for the stream and raises KcoreError if the last single-graph or batched call on it
    reported a device failure (kcore_check)."""
    _check(_lib.kcore_check(_stream_ptr(stream)), "kcore_check")


class Server:
    """Continuous-batching server over host graphs (see kcore.h, Serving)."""

    def __init__(self, device: int = 0, max_inflight: int = 0, max_batch_graphs: int = 0,
                 max_batch_vertices: int = 0, hbm_budget_bytes: int = 0,
                 max_request_vertices: int = 0, batch_wait_us: float = 0.0,
                 borrow_inputs: bool = False, reserve_vertices: int = 0, reserve_entries: int = 0,
                 fail_ticket: int = 0, max_large_inflight: int = 0, large_vertices: int = 0):
        cfg = ServerConfig()
        cfg.device = device
        cfg.max_inflight = max_inflight
        cfg.max_batch_graphs = max_batch_graphs
        cfg.max_large_inflight = max_large_inflight
        cfg.large_vertices = large_vertices
        cfg.max_batch_vertices = max_batch_vertices
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.max_request_vertices = max_request_vertices
        cfg.batch_wait_us = batch_wait_us
        cfg.borrow_inputs = 1 if borrow_inputs else 0
        cfg.reserve_vertices = reserve_vertices
        cfg.reserve_entries = reserve_entries
        cfg.fail_ticket = fail_ticket
        self._h = _lib.kcore_server_create(ctypes.byref(cfg))
        if not self._h:
            raise KcoreError(-1, "kcore_server_create", last_error())
        self._n = {}
        self._borrow = bool(borrow_inputs)
        self._held = {}

    def submit(self, offsets: np.ndarray, adj: np.ndarray) -> int:
        """Queues a host graph. With borrow_inputs the arrays must stay alive and unchanged until
        the result is taken (this object keeps a reference until then)."""
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        a = np.ascontiguousarray(adj, dtype=np.int32)
        n = off.shape[0] - 1
        t = ctypes.c_uint64(0)
        rc = _lib.kcore_submit(self._h, off.ctypes.data, a.ctypes.data if a.size else None, n,
                               ctypes.byref(t))
        _check(rc, "kcore_submit")
        self._n[t.value] = n
        if self._borrow:
            self._held[t.value] = (off, a)
        return t.value

    def poll(self, ticket: int):
        """(status, coreness or None, stats dict or None); status is KCORE_OK or KCORE_PENDING."""
        n = self._n.get(ticket, 0)
        out = np.empty(n, dtype=np.int32)
        st = RequestStats()
        rc = _lib.kcore_poll(self._h, ticket, out.ctypes.data if n else None, ctypes.byref(st))
        if rc == KCORE_PENDING:
            return rc, None, None
        self._n.pop(ticket, None)
        self._held.pop(ticket, None)
        _check(rc, "kcore_poll")
        return rc, out, st.as_dict()

    def wait(self, ticket: int, timeout_us: float = 0.0, with_stats: bool = False):
        n = self._n.get(ticket, 0)
        out = np.empty(n, dtype=np.int32)
        st = RequestStats()
        rc = _lib.kcore_wait(self._h, ticket, out.ctypes.data if n else None, ctypes.byref(st),
                             timeout_us)
        if rc == KCORE_PENDING:
            raise TimeoutError(f"ticket {ticket} not done after {timeout_us} us")
        self._n.pop(ticket, None)
        self._held.pop(ticket, None)
        _check(rc, "kcore_wait")
        return (out, st.as_dict()) if with_stats else out

    def cancel(self, ticket: int) -> int:
        return _lib.kcore_cancel(self._h, ticket)

    def now_us(self) -> float:
        return _lib.kcore_server_now_us(self._h)

    def close(self):
        if self._h:
            _lib.kcore_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
