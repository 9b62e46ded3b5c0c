#!/usr/bin/env python3
"""Benchmark of the MI355X k-core library.

Default (``--workload all``): the headline single-graph peel of the 16M-vertex Chung-Lu power-law
graph (gamma 2.1, ~1B directed entries, planted 5000-vertex G(n, 0.8) block; seed 3), reported as
peeled directed edges per second (GTEPS: adjacency entries m over the time of one decomposition,
graph resident in HBM) with its roofline position and the CPU oracle beside it; then every other
workload, each checked against the oracle, as keys of the same line:

  * ``rmat16``   R-MAT scale 16, edge factor 16 (single graph)
  * ``grid``     4096 x 4096 road-like grid (single graph, deep peel chains)
  * ``hcns``     staircase of coreness 20,000 (n = 40,000, 0.8B entries), with and without the
                 multi-bucket active set
  * ``batch``    4,096 graphs in one segmented CSR: one batched launch against a loop of the
                 single-graph call over the same graphs
  * ``serve``    Poisson arrivals at 20k requests/s (1% R-MAT scale 20), p50/p99 latency

    python bench.py [--steps K] [--warmup W] [--workload all|chunglu|rmat16|grid|hcns|batch|serve|kquery]

Prints exactly one JSON line. One GPU only: --gpus N with N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The serving workload gives each of its eight batch slots (three for large batches) a stream on a
# hardware queue of its own; HIP gives a process the number of queues GPU_MAX_HW_QUEUES says when
# it initialises (4 by default, and environments often set 4 explicitly), and streams beyond that
# share queues, so a small batch could wait behind a large one. The bench raises it to 16, with
# room for the queues the runtime uses itself, before anything initialises HIP.
os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "peeled directed edges/sec (GTEPS) + % HBM peak; batched graphs/sec & p99 latency"
HBM_PEAK_GBS = 8000.0
ORACLE_RUNS = 5          # timed oracle runs after one warm-up (the paper's protocol: mean of 5)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(n: int, m: int, st: dict) -> int:
    """Algorithmic bytes of one decomposition (the work bound of Thm. 3.1 priced in bytes): every
    adjacency entry read once (4m) with one read of its target's induced degree (4m), one 4-byte
    write per live decrement (a decrement landing on a vertex still above k: at most m/2), degree
    initialisation from the offsets (8(n+1)) into the induced degrees (4n), the offsets pair of each
    peeled vertex (16n), its coreness write and frontier write and read (12n), and 4 bytes per
    active-set slot scanned."""
    return (4 * m + 4 * m + 4 * st["live_decrements"] + 8 * (n + 1) + 4 * n + 16 * n + 12 * n
            + 4 * st["scanned"])


def host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def timed_calls(fn, steps: int, warmup: int):
    """Runs fn() warmup times, then steps times between HIP events recorded on the current
    stream (the stream the library launches on). Returns (wall ms per call, per-call event ms)."""
    import torch
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return (t2 - t1) * 1000.0 / steps, [e0.elapsed_time(e1) for e0, e1 in evs]


def summary(per):
    return {"mean": round(statistics.fmean(per), 4), "median": round(statistics.median(per), 4),
            "min": round(min(per), 4), "max": round(max(per), 4)}


def oracle_timing(h_off, h_adj, runs: int = ORACLE_RUNS):
    """The oracle (sequential Batagelj-Zaversnik, one host thread): one warm-up, then `runs`
    timed runs. Returns (coreness of the last run, list of seconds)."""
    import numpy as np
    import oracle
    core = np.empty(len(h_off) - 1, dtype=np.int32)
    secs = oracle.time_bz(h_off, h_adj, repeats=runs + 1, core_out=core)
    return core, secs[1:]


def cpu_baseline_entry(m: int, secs, sample: str) -> dict:
    med = statistics.median(secs)
    return {"value": round(m / med / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": sample, "median_s": round(med, 4), "mean_s": round(statistics.fmean(secs), 4),
            "runs": len(secs), "warmup_runs": 1, **host_info()}


def release():
    import torch
    import paper_2502_08042_amd as K
    torch.cuda.synchronize()
    K.release_workspaces()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------------------------
# single graph
# ---------------------------------------------------------------------------------------------
def build_workload(name: str):
    import torch
    import graphgen as gg
    if name == "chunglu":
        import graphgen.gpu as gp
        off, adj = gp.config_chung_lu_device()
        return off, adj, ("Chung-Lu n=2^24 gamma=2.1 32n endpoint pairs, degree cap 1e6, planted "
                          "5000-vertex G(n,0.8) block, symmetric int32 CSR, seed 3")
    if name == "hcns":
        import graphgen.gpu as gp
        off, adj = gp.hcns_device(20000)
        return off, adj, ("staircase of coreness K=20000: clique on K+1 vertices plus u_i adjacent "
                          "to clique vertices 0..i-1 (n=40000, 0.8B entries)")
    if name == "grid":
        g = gg.config_grid4096()
        desc = "road-like grid 4096x4096, 5% edges deleted, 1% unit-square diagonals, seed 2"
    elif name == "rmat16":
        g = gg.config_rmat16()
        desc = "RMAT scale 16 edge factor 16 a=.57 b=.19 c=.19, symmetrized, dedup'd, seed 1"
    else:
        raise ValueError(name)
    return torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda(), desc


def tuned_for(off, batched=False, explicit=None):
    """The autotuner's cached options for this device and the graph's class (explicit options
    win), and the class name."""
    import paper_2502_08042_amd.autotune as A
    opts = {} if explicit else A.tuned_options(off, batched=batched)
    return opts, A.workload_class(off, batched=batched)


def measure_single(off, adj, steps, warmup, mode="auto", **tuning):
    """Times kcore_decompose on a resident graph with the autotuner's options for its class (when
    the cache has them and no option is given). Returns (result dict, stats, coreness tensor)."""
    import torch
    import paper_2502_08042_amd as K
    n, m = off.numel() - 1, adj.numel()
    auto, cls = tuned_for(off, explicit=tuning)
    tuning = {**auto, **tuning}
    out = torch.empty(n, dtype=torch.int32, device=off.device)
    K.decompose(off, adj, out, mode=mode, **tuning)  # workspace allocation, outside the timing
    _, st = K.decompose(off, adj, out, mode=mode, stats=True, **tuning)
    wall_ms, per = timed_calls(lambda: K.decompose(off, adj, out, mode=mode, **tuning), steps, warmup)
    K.check()  # device status of the timed calls
    ev = summary(per)
    B = alg_bytes(n, m, st)
    res = {"n": n, "m": m, "mode": mode, "ms_per_step": round(wall_ms, 4), "event_ms": ev,
           "gteps": round(m / (ev["median"] / 1000.0) / 1e9, 4),
           "kmax": st["kmax"], "rounds": st["rounds"], "subrounds": st["subrounds"],
           "barriers": st["barriers"], "tail_vertices": st["tail_vertices"],
           "live_decrements": st["live_decrements"], "scanned": st["scanned"],
           "bucket_inserts": st["bucket_inserts"],
           "alg_bytes": B, "hbm_frac": round(B / (ev["mean"] / 1000.0) / 1e9 / HBM_PEAK_GBS, 5)}
    res["options"] = tuning
    res["workload_class"] = cls
    res["tuned"] = bool(auto)
    return res, st, out


def bench_chunglu(args):
    """The headline: one decomposition of the Chung-Lu graph per step."""
    import numpy as np
    import torch
    t0 = time.time()
    off, adj, desc = build_workload("chunglu")
    n, m = off.numel() - 1, adj.numel()
    log(f"[bench] chunglu: n={n} m={m} built in {time.time() - t0:.1f}s")
    r, st, out = measure_single(off, adj, args.steps, args.warmup, mode=args.mode)
    log(f"[bench] chunglu stats {json.dumps(st)}")
    ev = r["event_ms"]
    B = r["alg_bytes"]
    achieved = B / (ev["mean"] / 1000.0) / 1e9
    res = {
        "metric": METRIC, "value": round(m / (r["ms_per_step"] / 1000.0) / 1e9, 4), "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "m": m, "mode": args.mode, "kmax": r["kmax"],
                   "rounds": r["rounds"], "subrounds": r["subrounds"], "barriers": r["barriers"],
                   "tail_vertices": r["tail_vertices"], "options": r["options"],
                   "tuned": r["tuned"], "workload_class": r["workload_class"]},
        "gpu_event_ms": ev,
        # one decomposition = the persistent peel kernel, then the single-workgroup tail kernel on
        # the last live vertices (plus two tiny set-up kernels), all inside the events
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic_from_profile("peel_kernels_chunglu_traffic.txt", args.mode),
                     "alg_bytes_per_launch": B, "live_decrements": r["live_decrements"],
                     "scanned": r["scanned"], "kernel": "peel_kernel + tail_kernel",
                     "kernel_ms_per_launch": ev["mean"]},
    }
    if args.workload == "all":
        # the same graph with the multi-bucket active set (from n/8 live vertices at k >= 16)
        rb, _, outb = measure_single(off, adj, min(args.steps, 5), 1, mode=args.mode, buckets=n // 8)
        res["with_buckets"] = {k: rb[k] for k in ("ms_per_step", "event_ms", "gteps", "rounds", "barriers",
                                                  "scanned", "bucket_inserts", "tail_vertices", "hbm_frac")}
        res["with_buckets"]["options"] = {"buckets": n // 8}
        res["with_buckets"]["same_coreness"] = bool(torch.equal(outb, out))
        del outb
    if not args.no_cpu_baseline:
        h_off, h_adj = off.cpu().numpy(), adj.cpu().numpy()
        log(f"[bench] chunglu oracle: 1 warm-up + {ORACLE_RUNS} runs on one core")
        core, secs = oracle_timing(h_off, h_adj)
        res["cpu_baseline"] = cpu_baseline_entry(
            m, secs, f"the whole graph, 1 warm-up + {len(secs)} timed runs of the sequential oracle "
            f"(median {statistics.median(secs):.2f} s)")
        res["parity"] = bool(np.array_equal(out.cpu().numpy(), core))
    del off, adj, out
    release()
    return res


def bench_single_config(name, args, steps, warmup):
    """One of the other single-graph workloads: timing, counters and parity with the oracle."""
    import numpy as np
    t0 = time.time()
    off, adj, desc = build_workload(name)
    n, m = off.numel() - 1, adj.numel()
    log(f"[bench] {name}: n={n} m={m} built in {time.time() - t0:.1f}s")
    r, st, out = measure_single(off, adj, steps, warmup, mode=args.mode)
    r["workload"] = desc
    if name == "hcns":
        # the construction fixes every coreness: u_i has coreness i and the clique K
        K_ = n // 2
        want = np.concatenate([np.full(K_ + 1, K_, dtype=np.int32), np.arange(1, K_, dtype=np.int32)])
        r["parity"] = bool(np.array_equal(out.cpu().numpy(), want))
        r["parity_against"] = "closed form of the construction"
        rb, _, outb = measure_single(off, adj, steps, warmup, mode=args.mode, buckets=1 << 30)
        r["with_buckets"] = {k: rb[k] for k in ("ms_per_step", "event_ms", "gteps", "rounds",
                                                "barriers", "scanned", "bucket_inserts",
                                                "tail_vertices", "hbm_frac")}
        r["with_buckets"]["parity"] = bool(np.array_equal(outb.cpu().numpy(), want))
        r["buckets_speedup"] = round(r["event_ms"]["median"] / rb["event_ms"]["median"], 3)
        del outb
    else:
        h_off, h_adj = off.cpu().numpy(), adj.cpu().numpy()
        core, secs = oracle_timing(h_off, h_adj)
        r["parity"] = bool(np.array_equal(out.cpu().numpy(), core))
        r["cpu_oracle"] = {"median_s": round(statistics.median(secs), 5),
                           "gteps": round(m / statistics.median(secs) / 1e9, 5), "runs": len(secs)}
    del off, adj, out
    release()
    return r


def traffic_from_profile(fname: str, mode: str):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs kept in profiles/
    (calibrated against a plain copy), valid only for the kernel source they were taken on."""
    tfile = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(tfile):
        return None
    with open(tfile) as f:
        tj = json.load(f)
    if tj.get("kernel_source_sha") == kernel_sha() and tj.get("mode", mode) == mode:
        return tj.get("bytes_per_launch")
    return None


# ---------------------------------------------------------------------------------------------
# batched and serving
# ---------------------------------------------------------------------------------------------
def bench_batch(args, steps, warmup):
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
    topts, cls = tuned_for(off, batched=True)
    K.decompose_batched(vptr, off, adj, out, **topts)
    _, st = K.decompose_batched(vptr, off, adj, out, stats=True, **topts)
    want = oracle.bz(b.offsets, b.adj)
    parity = bool(np.array_equal(out.cpu().numpy(), want))
    wall_ms, per = timed_calls(lambda: K.decompose_batched(vptr, off, adj, out, **topts), steps, warmup)
    K.check()
    ev = summary(per)
    # the same graphs, one single-graph call each (local ids)
    parts = []
    for g in range(G):
        lo, hi = int(b.vptr[g]), int(b.vptr[g + 1])
        e0_, e1_ = int(b.offsets[lo]), int(b.offsets[hi])
        parts.append((off[lo:hi + 1] - e0_, adj[e0_:e1_] - lo, out[lo:hi]))
    for o_, a_, c_ in parts[:64]:
        K.decompose(o_, a_, c_)
    out.fill_(-1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for o_, a_, c_ in parts:
        K.decompose(o_, a_, c_)
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t3) * 1000.0
    K.check()
    loop_parity = bool(np.array_equal(out.cpu().numpy(), want))
    B = alg_bytes(V, m, st)
    res = {"workload": "4096 graphs, lognormal n (median 2000, sigma 1, 100..100000), even ER avg "
                       "deg 8 / odd RMAT 8n draws, one segmented CSR, seed 4",
           "graphs": G, "vertices": V, "m": m, "steps": steps, "ms_per_step": round(wall_ms, 4),
           "event_ms": ev, "graphs_per_s": round(G / (wall_ms / 1000.0), 1),
           "gteps": round(m / (wall_ms / 1000.0) / 1e9, 4),
           "per_graph_loop_ms": round(ms_loop, 3), "speedup_vs_loop": round(ms_loop / wall_ms, 2),
           "parity": parity and loop_parity, "options": topts, "tuned": bool(topts), "workload_class": cls,
           "roofline": {"bound": "hbm", "achieved": round(B / (ev["mean"] / 1000.0) / 1e9, 2),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(B / (ev["mean"] / 1000.0) / 1e9 / HBM_PEAK_GBS, 5),
                        "traffic": traffic_from_profile("batched_kernel_batch4096_traffic.txt", "auto"),
                        "alg_bytes_per_launch": B, "kernel": "batched_kernel",
                        "kernel_ms_per_launch": ev["mean"]}}
    # where the launch's time goes: the same call on the graphs of one size class alone
    ns = np.diff(b.vptr)
    res["by_size"] = {}
    for name, sel in (("n<=9152 (LDS-resident)", ns <= 9152), ("n>9152", ns > 9152), ("n>20000", ns > 20000)):
        sv, so, sa = sub_batch(b, np.flatnonzero(sel))
        sc = torch.empty(int(sv[-1]), dtype=torch.int32, device="cuda")
        t = [torch.from_numpy(x).cuda() for x in (sv, so, sa)]
        K.decompose_batched(*t, sc, **topts)
        _, per_s = timed_calls(lambda: K.decompose_batched(*t, sc, **topts), 5, 1)
        res["by_size"][name] = {"graphs": int(sel.sum()), "entries": int(so[-1]),
                                "event_ms_median": summary(per_s)["median"]}
        del t, sc
    K.check()
    del parts, vptr, off, adj, out
    release()
    return res


def sub_batch(b, sel):
    """Segmented CSR (vptr, offsets, adj with ids renumbered) of the graphs `sel` of batch b."""
    import numpy as np
    vp, offs, adjs, e0 = [0], [np.zeros(1, np.int64)], [], 0
    for g in sel:
        v0, v1 = int(b.vptr[g]), int(b.vptr[g + 1])
        o = b.offsets[v0:v1 + 1].astype(np.int64)
        adjs.append((b.adj[o[0]:o[-1]].astype(np.int64) - v0 + vp[-1]).astype(np.int32))
        offs.append(o[1:] - o[0] + e0)
        e0 += int(o[-1] - o[0])
        vp.append(vp[-1] + (v1 - v0))
    return (np.array(vp, np.int64), np.concatenate(offs),
            np.concatenate(adjs) if adjs else np.zeros(0, np.int32))


def bench_serve(args, seconds: float = 5.0, rate: float = 20000.0, warm: float = 1.0, **server_kw):
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
    # a slot per two hardware queues of the process, at most eight (streams beyond the queues share
    # them, and a small batch would wait behind a large one), three of eight for large batches;
    # slot buffers sized up front for full small batches
    server_kw.setdefault("max_inflight", max(2, min(8, int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) // 2)))
    mi = server_kw["max_inflight"]
    server_kw.setdefault("max_large_inflight", 3 if mi >= 8 else (2 if mi >= 3 else 1))
    srv = K.Server(device=0, hbm_budget_bytes=64 << 30, max_batch_vertices=1 << 25,
                   borrow_inputs=True, reserve_vertices=1 << 24, reserve_entries=160 << 20, **server_kw)
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
            results[i] = (out, (rs.submit_us, rs.admit_us, rs.launch_us, rs.done_us, rs.batch_id,
                                rs.batch_graphs))
        done_evt.set()

    # the submitting loop and the collector share the interpreter lock; a short switch interval
    # keeps the submitter on schedule (its lag behind the arrival times is reported apart)
    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
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
        rc = lib.kcore_submit(srv._h, g.offsets.ctypes.data, g.adj.ctypes.data, g.n, ctypes.byref(tk))
        if rc != 0:
            raise K.KcoreError(rc, "kcore_submit", K.last_error())
        tickets[i] = tk.value
    done_evt.wait()
    sys.setswitchinterval(switch)
    srv.close()
    lat = np.empty(nreq)
    late = np.empty(nreq)    # scheduled arrival -> submitted (the client's own lag)
    wait = np.empty(nreq)    # submitted -> admitted into a batch (the server's queue)
    dev = np.empty(nreq)     # batch enqueued -> result visible (copies and the peel on the device)
    ok = True
    last_done = 0.0
    batches = {}
    for i in range(nreq):
        core, (submit_us, admit_us, launch_us, done_us, bid, bg) = results[i]
        lat[i] = done_us - (t0 + arrivals[i])
        late[i] = submit_us - (t0 + arrivals[i])
        wait[i] = admit_us - submit_us
        dev[i] = done_us - launch_us
        want = want_big[pick[i] % 2] if is_big[i] else want_small[pick[i]]
        ok = ok and bool(np.array_equal(core, want))
        if arrivals[i] < warm * 1e6:
            continue
        last_done = max(last_done, done_us)
        batches[bid] = (bool(is_big[i]), bg, launch_us - admit_us, done_us - launch_us)
    meas = arrivals >= warm * 1e6
    nmeas = int(meas.sum())
    lat, late, wait, dev, is_big = lat[meas], late[meas], wait[meas], dev[meas], is_big[meas]
    span_s = (last_done - (t0 + warm * 1e6)) / 1e6
    per_class = {}
    for cls, name in ((False, "small"), (True, "large")):
        b = np.array([x[1:] for x in batches.values() if x[0] == cls], dtype=np.float64)
        if len(b):
            per_class[name] = {"batches": len(b), "mean_graphs": round(float(b[:, 0].mean()), 1),
                               "mean_pack_ms": round(float(b[:, 1].mean()) / 1000, 3),
                               "mean_launch_to_done_ms": round(float(b[:, 2].mean()) / 1000, 3)}
    del keep
    release()
    return {
        "workload": f"serving: Poisson {rate:.0f} req/s, {warm:g}s warm-up then {seconds:g}s measured, "
                    "graphs from the batched distribution, 1% R-MAT scale 20 edge factor 16",
        "requests": nmeas, "offered_per_s": rate, "graphs_per_s": round(nmeas / span_s, 1),
        "span_s": round(span_s, 3),
        "p50_ms": round(float(np.percentile(lat, 50)) / 1000, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) / 1000, 3),
        "p99_small_ms": round(float(np.percentile(lat[~is_big], 99)) / 1000, 3),
        "p99_large_ms": round(float(np.percentile(lat[is_big], 99)) / 1000, 3) if is_big.any() else None,
        "p99_small_submit_lag_ms": round(float(np.percentile(late[~is_big], 99)) / 1000, 3),
        "p99_small_wait_ms": round(float(np.percentile(wait[~is_big], 99)) / 1000, 3),
        "p99_small_device_ms": round(float(np.percentile(dev[~is_big], 99)) / 1000, 3),
        "batches": per_class, "parity": ok,
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
    K.kcore_subgraph(off, adj, k, out)
    wall_ms, per = timed_calls(lambda: K.kcore_subgraph(off, adj, k, out), args.steps, args.warmup)
    K.check()
    got = out.cpu().numpy()
    want = (oracle.bz(off.cpu().numpy(), adj.cpu().numpy()) >= k).astype(np.int32)
    return {"workload": f"maximum {k}-core subgraph of: {desc}", "n": n, "m": m, "k": k,
            "ms_per_step": round(wall_ms, 4), "event_ms": summary(per),
            "gteps": round(m / (wall_ms / 1000.0) / 1e9, 4),  # (input entries per second)
            "core_size": int(got.sum()), "parity": bool(np.array_equal(got, want))}


def kernel_sha() -> str:
    """Hash of the kernel sources (the device code and the constants it is built with)."""
    import hashlib
    h = hashlib.sha1()
    for name in ("kcore_device.hip", "kcore_internal.h"):
        with open(os.path.join(ROOT, "paper_2502_08042_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def wrap_single(name, r, args):
    """A single-workload run printed on its own (``--workload X``)."""
    # batched and serving runs are quoted in graphs per second, single graphs in GTEPS
    per_graph = name in ("batch", "serve")
    return {"metric": METRIC, "value": r.get("graphs_per_s") if per_graph else r.get("gteps"),
            "unit": "graphs/s" if per_graph else "GTEPS",
            "n_gpus": 1, "steps": r.get("steps", args.steps), "warmup": args.warmup,
            "ms_per_step": r.get("ms_per_step"), "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": r.get("workload", name)}, name: r}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="all",
                    choices=["all", "chunglu", "grid", "rmat16", "hcns", "batch", "serve", "kquery"])
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
    # the secondary workloads use at most 10 timed steps each, so the whole run stays short
    sub_steps, sub_warm = min(args.steps, 10), min(args.warmup, 2)
    if args.workload == "chunglu":
        res = bench_chunglu(args)
    elif args.workload == "all":
        res = bench_chunglu(args)
        cfg = {}
        for name in ("rmat16", "grid", "hcns"):
            cfg[name] = bench_single_config(name, args, sub_steps if name != "hcns" else min(sub_steps, 3),
                                            sub_warm if name != "hcns" else 1)
            log(f"[bench] {name}: {json.dumps(cfg[name])}")
        cfg["batch"] = bench_batch(args, sub_steps, sub_warm)
        log(f"[bench] batch: {json.dumps(cfg['batch'])}")
        cfg["serve"] = bench_serve(args)
        log(f"[bench] serve: {json.dumps(cfg['serve'])}")
        res["configs"] = cfg
        res["parity_all"] = bool(res.get("parity", True)) and all(
            bool(c.get("parity")) for c in cfg.values())
    elif args.workload in ("rmat16", "grid", "hcns"):
        res = wrap_single(args.workload, bench_single_config(args.workload, args, args.steps, args.warmup), args)
    elif args.workload == "batch":
        res = wrap_single("batch", bench_batch(args, args.steps, args.warmup), args)
    elif args.workload == "serve":
        res = wrap_single("serve", bench_serve(args), args)
    else:
        res = wrap_single("kquery", bench_kquery(args), args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
