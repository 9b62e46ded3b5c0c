#!/usr/bin/env python3
"""Benchmark of the MI355X k-core library.

Default: single-graph peel of the 16M-vertex Chung-Lu power-law graph (gamma 2.1, ~1B directed
entries, planted 5000-vertex G(n, 0.8) block; seed 3) — the headline workload. Reports peeled
directed edges per second (GTEPS: adjacency entries m divided by the time of one decomposition,
graph resident in HBM), the roofline position of the peel kernel and the CPU oracle's rate on the
same graph.

    python bench.py [--steps K] [--warmup W] [--workload chunglu|grid|rmat16|batch|serve|kquery]

Prints exactly one JSON line. One GPU only: --gpus N with N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "peeled directed edges/sec (GTEPS) + % HBM peak; batched graphs/sec & p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(n: int, m: int, st: dict) -> int:
    """Algorithmic bytes of one decomposition: adjacency read once (4m), one liveness probe per
    entry (4m), one 4-byte read-modify-write per applied decrement, whether applied one at a time
    or as a combined count (8 each), degree init from offsets (8(n+1)) and induced-degree init
    (4n), the offsets pair of each peeled vertex (16n), coreness write plus frontier write and read
    (12n), and 4 bytes per scanned active-set slot."""
    return (4 * m + 4 * m + 8 * (st["decrements"] + st["combined"]) + 8 * (n + 1) + 4 * n
            + 16 * n + 12 * n + 4 * st["scanned"])


def build_workload(name: str):
    import numpy as np
    import torch
    import graphgen as gg
    if name == "chunglu":
        import graphgen.gpu as gp
        off, adj = gp.config_chung_lu_device()
        desc = ("Chung-Lu n=2^24 gamma=2.1 32n endpoint pairs, degree cap 1e6, planted 5000-vertex "
                "G(n,0.8) block, symmetric int32 CSR, seed 3")
        return off, adj, desc
    if name == "grid":
        g = gg.config_grid4096()
        desc = "road-like grid 4096x4096, 5% edges deleted, 1% unit-square diagonals, seed 2"
    elif name == "rmat16":
        g = gg.config_rmat16()
        desc = "RMAT scale 16 edge factor 16 a=.57 b=.19 c=.19, symmetrized, seed 1"
    else:
        raise ValueError(name)
    return (torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda(), desc)


def bench_single(args):
    import numpy as np
    import torch
    import paper_2502_08042_amd as K
    t0 = time.time()
    off, adj, desc = build_workload(args.workload)
    torch.cuda.synchronize()
    n, m = off.numel() - 1, adj.numel()
    log(f"[bench] workload {args.workload}: n={n} m={m} built in {time.time() - t0:.1f}s")
    out = torch.empty(n, dtype=torch.int32, device=off.device)
    for _ in range(args.warmup):
        K.decompose(off, adj, out, mode=args.mode)
    _, st = K.decompose(off, adj, out, mode=args.mode, stats=True)
    log(f"[bench] stats {json.dumps(st)}")
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        K.decompose(off, adj, out, mode=args.mode)
        e1.record(stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    per = [e0.elapsed_time(e1) for e0, e1 in evs]
    ms_step = (t2 - t1) * 1000.0 / args.steps
    avg_ms = sum(per) / len(per)
    value = m / (ms_step / 1000.0) / 1e9
    B = alg_bytes(n, m, st)
    achieved = B / (avg_ms / 1000.0) / 1e9
    # HBM bytes per decomposition (peel kernel + tail kernel) from the rocprofv3 FETCH_SIZE /
    # WRITE_SIZE runs (calibrated against a plain copy), valid only for the kernel source they were
    # taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"peel_kernels_{args.workload}_traffic.txt")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tj = json.load(f)
        if tj.get("kernel_source_sha") == kernel_sha() and tj.get("mode") == args.mode:
            traffic = tj.get("bytes_per_launch")
    res = {
        "metric": METRIC, "value": round(value, 4), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "m": m, "mode": args.mode,
                   "kmax": st["kmax"], "rounds": st["rounds"], "subrounds": st["subrounds"],
                   "barriers": st["barriers"], "tail_vertices": st["tail_vertices"]},
        # one decomposition = the persistent peel kernel, then the single-workgroup tail kernel on
        # the last live vertices (plus two tiny set-up kernels), all inside the events
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic, "alg_bytes_per_launch": B,
                     "kernel": "peel_kernel + tail_kernel",
                     "kernel_ms_per_launch": round(avg_ms, 4)},
    }
    if not args.no_cpu_baseline:
        # the same oracle run also checks the last decomposition's coreness, vertex by vertex
        res["cpu_baseline"], res["parity"] = cpu_baseline(off, adj, m, out)
    return res


def cpu_baseline(off, adj, m, out_dev):
    """The oracle (sequential Batagelj-Zaversnik, one host thread) on the same graph, once."""
    import numpy as np
    import oracle
    t0 = time.time()
    h_off = off.cpu().numpy()
    h_adj = adj.cpu().numpy()
    log(f"[bench] host copy {time.time() - t0:.1f}s; running the oracle once on one core")
    core = np.empty(len(h_off) - 1, dtype=np.int32)
    secs = oracle.time_bz(h_off, h_adj, repeats=1, core_out=core)[0]
    return {"value": round(m / secs / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"whole graph, one run of the sequential oracle ({secs:.1f} s)"}, \
        bool(np.array_equal(out_dev.cpu().numpy(), core))


def bench_batch(args):
    """4096 lognormal-sized graphs in one segmented CSR: one batched launch vs a loop of the
    single-graph call over the same graphs."""
    import numpy as np
    import torch
    import graphgen as gg
    import oracle
    import paper_2502_08042_amd as K
    t0 = time.time()
    b = gg.config_batch()
    G, V, m = len(b.vptr) - 1, b.n, b.m
    vptr = torch.from_numpy(b.vptr).cuda()
    off = torch.from_numpy(b.offsets).cuda()
    adj = torch.from_numpy(b.adj).cuda()
    log(f"[bench] batch G={G} V={V} m={m} built in {time.time() - t0:.1f}s")
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        K.decompose_batched(vptr, off, adj, out)
    _, st = K.decompose_batched(vptr, off, adj, out, stats=True)
    want = oracle.bz(b.offsets, b.adj)
    parity = bool(np.array_equal(out.cpu().numpy(), want))
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        K.decompose_batched(vptr, off, adj, out)
        e1.record(stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms_batch = (t2 - t1) * 1000.0 / args.steps
    kern_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / args.steps
    # the same graphs, one single-graph call each (local ids)
    parts = []
    for g in range(G):
        lo, hi = int(b.vptr[g]), int(b.vptr[g + 1])
        e0_, e1_ = int(b.offsets[lo]), int(b.offsets[hi])
        parts.append((off[lo:hi + 1] - e0_, adj[e0_:e1_] - lo, out[lo:hi], e1_ - e0_))
    for o_, a_, c_, mm in parts[:64]:
        K.decompose(o_, a_, c_)
    out.fill_(-1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for o_, a_, c_, mm in parts:
        K.decompose(o_, a_, c_)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    ms_loop = (t4 - t3) * 1000.0
    loop_parity = bool(np.array_equal(out.cpu().numpy(), want))
    B = alg_bytes(V, m, st)
    # HBM bytes per batched launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs (calibrated
    # against a plain copy), valid only for the kernel source they were taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "batched_kernel_batch4096_traffic.txt")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tj = json.load(f)
        if tj.get("kernel_source_sha") == kernel_sha():
            traffic = tj.get("bytes_per_launch")
    return {
        "metric": METRIC, "value": round(G / (ms_batch / 1000.0), 1), "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_batch, 4),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "4096 graphs, lognormal n (median 2000, sigma 1, 100..100000), even "
                   "ER avg deg 8 / odd RMAT 8n draws, one segmented CSR, seed 4",
                   "graphs": G, "vertices": V, "m": m},
        "batched_gteps": round(m / (ms_batch / 1000.0) / 1e9, 4),
        "per_graph_loop_ms": round(ms_loop, 3), "speedup_vs_loop": round(ms_loop / ms_batch, 2),
        "parity": parity and loop_parity,
        "roofline": {"bound": "hbm", "achieved": round(B / (kern_ms / 1000.0) / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(B / (kern_ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "alg_bytes_per_launch": B, "kernel": "batched_kernel",
                     "kernel_ms_per_launch": round(kern_ms, 4)},
    }


def bench_serve(args, seconds: float = 5.0, rate: float = 20000.0, warm: float = 1.0):
    """Open-loop Poisson arrivals (20k req/s) of graphs from the batched distribution, 1% replaced
    by R-MAT scale 20 edge factor 16; latency = result visible - scheduled arrival. The first
    `warm` seconds of arrivals (buffers growing to their working sizes) are served but not counted."""
    import threading
    import numpy as np
    import graphgen as gg
    import oracle
    import paper_2502_08042_amd as K
    import torch
    pool = gg.batch(512, 5, first_graph=100000)
    small = [pool.subgraph(g) for g in range(512)]
    big = [gg.rmat(20, 16, 50 + i) for i in range(2)]

    def pinned(g):
        # request graphs live in pinned host memory: the server borrows them and copies large ones
        # to the device by DMA
        o = torch.from_numpy(g.offsets).pin_memory()
        a = torch.from_numpy(g.adj).pin_memory()
        return gg.Graph(o.numpy(), a.numpy(), None, g.name), (o, a)

    keep = []
    small2, big2 = [], []
    for g in small:
        h, t = pinned(g)
        small2.append(h)
        keep.append(t)
    for g in big:
        h, t = pinned(g)
        big2.append(h)
        keep.append(t)
    small, big = small2, big2
    want_small = [oracle.bz(g.offsets, g.adj) for g in small]
    want_big = [oracle.bz(g.offsets, g.adj) for g in big]
    nreq = int((seconds + warm) * rate)
    u = gg.uniform(5, 91, 0, 3 * nreq)
    gaps = -np.log1p(-u[:nreq]) / rate
    arrivals = np.cumsum(gaps) * 1e6  # us
    is_big = u[nreq:2 * nreq] < 0.01
    pick = (u[2 * nreq:] * 512).astype(np.int64)
    log(f"[bench] serving {nreq} requests over {arrivals[-1] / 1e6:.1f}s, {int(is_big.sum())} large")
    # four slots, one per hardware queue of the process (streams beyond that share queues, and a
    # small batch would wait behind a large one); slot buffers sized up front for full small batches
    srv = K.Server(device=0, max_inflight=4, hbm_budget_bytes=64 << 30, max_batch_vertices=1 << 25,
                   borrow_inputs=True, reserve_vertices=1 << 24, reserve_entries=160 << 20)
    tickets = [None] * nreq
    results = {}
    done_evt = threading.Event()

    lib = K.lib()
    n_of = [None] * nreq

    def collector():
        # straight through the C ABI with preallocated outputs: the client's own per-request cost
        # must stay well below the server's
        rs = K.RequestStats()
        for i in range(nreq):
            while tickets[i] is None:
                time.sleep(0.0002)
            out = np.empty(n_of[i], dtype=np.int32)
            rc = lib.kcore_wait(srv._h, tickets[i], out.ctypes.data if n_of[i] else None,
                                ctypes.byref(rs), 0.0)
            if rc != 0:
                raise K.KcoreError(rc, "kcore_wait", K.last_error())
            results[i] = (out, (rs.admit_us, rs.launch_us, rs.done_us, rs.batch_id, rs.batch_graphs))
        done_evt.set()

    th = threading.Thread(target=collector, daemon=True)
    th.start()
    t0 = srv.now_us()
    tk = ctypes.c_uint64(0)
    for i in range(nreq):
        due = t0 + arrivals[i]
        while srv.now_us() < due:
            pass
        g = big[pick[i] % 2] if is_big[i] else small[pick[i]]
        n_of[i] = g.n
        # the inputs live in the pinned pool for the whole run (borrowed, never copied on submit)
        rc = lib.kcore_submit(srv._h, g.offsets.ctypes.data, g.adj.ctypes.data, g.n, ctypes.byref(tk))
        if rc != 0:
            raise K.KcoreError(rc, "kcore_submit", K.last_error())
        tickets[i] = tk.value
    done_evt.wait()
    srv.close()
    lat = np.empty(nreq)
    ok = True
    last_done = 0.0
    batches = {}
    for i in range(nreq):
        core, (admit_us, launch_us, done_us, bid, bg) = results[i]
        lat[i] = done_us - (t0 + arrivals[i])
        want = want_big[pick[i] % 2] if is_big[i] else want_small[pick[i]]
        ok = ok and bool(np.array_equal(core, want))
        if arrivals[i] < warm * 1e6:
            continue
        last_done = max(last_done, done_us)
        batches[bid] = (bool(is_big[i]), bg, launch_us - admit_us, done_us - launch_us)
    meas = arrivals >= warm * 1e6
    nmeas = int(meas.sum())
    lat, is_big = lat[meas], is_big[meas]
    span_s = (last_done - (t0 + warm * 1e6)) / 1e6
    per_class = {}
    for cls, name in ((False, "small"), (True, "large")):
        b = np.array([x[1:] for x in batches.values() if x[0] == cls], dtype=np.float64)
        if len(b):
            per_class[name] = {"batches": len(b), "mean_graphs": round(float(b[:, 0].mean()), 1),
                               "mean_pack_ms": round(float(b[:, 1].mean()) / 1000, 3),
                               "mean_launch_to_done_ms": round(float(b[:, 2].mean()) / 1000, 3)}
    return {
        "metric": METRIC, "value": round(nmeas / span_s, 1), "unit": "graphs/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(span_s * 1000, 1), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"serving: Poisson {rate:.0f} req/s, {warm:g}s warm-up then {seconds:g}s "
                   "measured, graphs from the batched distribution, 1% R-MAT scale 20 edge factor 16",
                   "requests": nmeas},
        "p50_ms": round(float(np.percentile(lat, 50)) / 1000, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) / 1000, 3),
        "p99_small_ms": round(float(np.percentile(lat[~is_big], 99)) / 1000, 3),
        "p99_large_ms": round(float(np.percentile(lat[is_big], 99)) / 1000, 3) if is_big.any() else None,
        "batches": per_class,
        "parity": ok,
    }


def bench_kquery(args, k: int = 1000):
    """Maximum k-core subgraph (one peeling round at k - 1) of the Chung-Lu graph; membership checked
    against the oracle's coreness."""
    import numpy as np
    import torch
    import oracle
    import paper_2502_08042_amd as K
    off, adj, desc = build_workload("chunglu")
    torch.cuda.synchronize()
    n, m = off.numel() - 1, adj.numel()
    out = torch.empty(n, dtype=torch.int32, device=off.device)
    for _ in range(args.warmup):
        K.kcore_subgraph(off, adj, k, out)
    _, st = K.kcore_subgraph(off, adj, k, out, stats=True)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        K.kcore_subgraph(off, adj, k, out)
        e1.record(stream)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t1) * 1000.0 / args.steps
    kern_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / args.steps
    got = out.cpu().numpy()
    want = (oracle.bz(off.cpu().numpy(), adj.cpu().numpy()) >= k).astype(np.int32)
    return {
        "metric": METRIC, "value": round(m / (ms_step / 1000.0) / 1e9, 4), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"maximum {k}-core subgraph of: {desc}", "n": n, "m": m, "k": k,
                   "core_size": int(got.sum()), "peeled": int(n - got.sum())},
        "kernel_ms_per_launch": round(kern_ms, 4), "parity": bool(np.array_equal(got, want)),
    }


def kernel_sha() -> str:
    """Hash of the kernel sources (the device code and the constants it is built with)."""
    import hashlib
    h = hashlib.sha1()
    for name in ("kcore_device.hip", "kcore_internal.h"):
        with open(os.path.join(ROOT, "paper_2502_08042_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chunglu", choices=["chunglu", "grid", "rmat16", "batch", "serve", "kquery"])
    ap.add_argument("--mode", default="auto", choices=["auto", "levelsync", "chained", "sampling", "offline"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the single-graph, batched "
              "and serving paths each run on one device", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        res = bench_batch(args)
    elif args.workload == "serve":
        res = bench_serve(args)
    elif args.workload == "kquery":
        res = bench_kquery(args)
    else:
        res = bench_single(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
