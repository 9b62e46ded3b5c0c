"""Autotuner for the library's launch and tiling parameters.

The peel kernels expose their tile and workgroup sizes and their phase thresholds as
``kcore_options`` fields (see include/kcore.h). Which values are fastest depends on the device and
on the shape of the graph, so this module sweeps them on a representative input, one parameter at
a time from the library defaults (coordinate descent, two passes), times every candidate with the
library's own device events (median of a few runs), and keeps a candidate only when its coreness
is identical to the default configuration's. The winners go to a JSON cache keyed by device and
workload class; ``tuned_options`` reads it back, and ``decompose(..., tuned=True)`` /
``decompose_batched(..., tuned=True)`` in the binding apply it.

Workload classes (from the CSR shape, computed with two reductions over ``offsets``):
``single/<size>/<density>/<skew>`` and ``batched/<size>``, where size is the power of four of the
vertex count, density bins the average degree (<= 8, <= 32, > 32) and skew says whether the
largest degree exceeds 64 times the average.

Command line (on a GPU machine)::

    python -m paper_2502_08042_amd.autotune [--workloads rmat16,grid,chunglu,hcns,batch] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "tuning", "cache.json")

# Candidate values of each option; 0 is the library default. Coordinate descent starts from all
# defaults and moves one option at a time.
SINGLE_SPACE = {
    "tile_edges": [0, 128, 512, 1024],
    "hub_degree": [0, 128, 512, 1024],
    "blocks_per_cu": [0, 1],
    "block_tiles": [0, 8, 128, -1],
    "block_queue": [0, 16, 256],
    "residual": [0, -1, "n/64", "n/1024"],
    "tail": [0, -1, "n/32", "n/2"],
    "buckets": [0, "n"],
    "combine_degree": [0, 256, 4096],
    "big_phase": [0, 4096, 65536],
    "local_budget": [0, 512, 4096],
    "async_frontier": [0, -1, 16384],
    "async_scan": [0, 65536],
}
BATCHED_SPACE = {
    "mode": ["levelsync", "chained"],
    "blocks_per_cu": [0, 1],
    "team_size": [0, 8, 16],
    "batch_teams": [0, -1, 200000],
}


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}-{p.multi_processor_count}cu"


def workload_class(offsets, batched: bool = False) -> str:
    """Class of a device CSR (int64 offsets[n+1]) from its size, mean and largest degree."""
    import torch
    n = offsets.numel() - 1
    size = 0 if n <= 1 else int(math.log(n, 4))
    if batched:
        return f"batched/{size}"
    if n <= 0:
        return "single/0/sparse/flat"
    deg = offsets[1:] - offsets[:-1]
    m = int(offsets[-1] - offsets[0])
    dmax = int(torch.max(deg))
    avg = m / n
    dens = "sparse" if avg <= 8 else ("medium" if avg <= 32 else "dense")
    skew = "skewed" if dmax > 64 * max(avg, 1.0) else "flat"
    return f"single/{size}/{dens}/{skew}"


def _resolve(opts: dict, n: int) -> dict:
    """Options with symbolic values (n/64, ...) turned into numbers for an n-vertex graph."""
    out = {}
    for k, v in opts.items():
        if isinstance(v, str) and v.startswith("n"):
            v = n if v == "n" else max(1, n // int(v.split("/")[1]))
            v = min(v, (1 << 31) - 1)
        out[k] = v
    return out


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned_options(offsets, batched: bool = False, path: str = DEFAULT_CACHE) -> dict:
    """Options the cache holds for this device and the graph's workload class ({} if none)."""
    cache = load_cache(path)
    ent = cache.get(device_key(), {}).get(workload_class(offsets, batched))
    if not ent:
        return {}
    # (only what differs from the library defaults)
    return {k: v for k, v in _resolve(ent["options"], offsets.numel() - 1).items()
            if v != 0 and v != "levelsync"}


def _time_single(off, adj, opts, reps):
    import paper_2502_08042_amd as K
    ms = []
    core = None
    for _ in range(reps):
        core, st = K.decompose(off, adj, stats=True, **opts)
        ms.append(st["ms"])
    return statistics.median(ms), core


def _time_batched(vptr, off, adj, opts, reps):
    import paper_2502_08042_amd as K
    ms = []
    core = None
    for _ in range(reps):
        core, st = K.decompose_batched(vptr, off, adj, stats=True, **opts)
        ms.append(st["ms"])
    return statistics.median(ms), core


def tune(space: dict, run, log=print, passes: int = 2):
    """Coordinate descent over `space` with run(opts) -> (ms, coreness tensor). A candidate whose
    coreness differs from the default configuration's is rejected (the result is exact, so any
    difference is a defect). Returns (best options, best ms, default ms, trials)."""
    import torch
    base = {k: v[0] for k, v in space.items()}
    ref_ms, ref = run(base)
    best, best_ms = dict(base), ref_ms
    trials = [{"options": dict(base), "ms": round(ref_ms, 4)}]
    log(f"[tune] default {base}: {ref_ms:.3f} ms")
    for _ in range(passes):
        moved = False
        for key, values in space.items():
            for v in values:
                if v == best[key]:
                    continue
                cand = dict(best)
                cand[key] = v
                ms, core = run(cand)
                same = bool(torch.equal(core, ref))
                trials.append({"options": dict(cand), "ms": round(ms, 4), "exact": same})
                log(f"[tune] {key}={v}: {ms:.3f} ms{'' if same else '  REJECTED: coreness differs'}")
                if same and ms < best_ms * 0.98:
                    best, best_ms, moved = cand, ms, True
        if not moved:
            break
    return best, best_ms, ref_ms, trials


def tune_single(off, adj, reps: int = 3, log=print):
    n = off.numel() - 1
    space = {k: [_resolve({k: v}, n)[k] for v in vals] for k, vals in SINGLE_SPACE.items()}
    # (the symbolic forms are what the cache stores, so that a class entry fits any size)
    best, best_ms, ref_ms, trials = tune(space, lambda o: _time_single(off, adj, o, reps), log)
    sym = {}
    for k, vals in SINGLE_SPACE.items():
        for v in vals:
            if _resolve({k: v}, n)[k] == best[k]:
                sym[k] = v
                break
    return sym, best_ms, ref_ms, trials


def tune_batched(vptr, off, adj, reps: int = 5, log=print):
    best, best_ms, ref_ms, trials = tune(BATCHED_SPACE, lambda o: _time_batched(vptr, off, adj, o, reps), log)
    return best, best_ms, ref_ms, trials


def _workloads(names):
    import torch
    import graphgen as gg
    for name in names:
        if name == "chunglu":
            import graphgen.gpu as gp
            off, adj = gp.config_chung_lu_device()
            yield name, False, (off, adj)
        elif name == "hcns":
            import graphgen.gpu as gp
            off, adj = gp.hcns_device(20000)
            yield name, False, (off, adj)
        elif name == "batch":
            b = gg.config_batch()
            yield name, True, tuple(torch.from_numpy(x).cuda() for x in (b.vptr, b.offsets, b.adj))
        else:
            g = {"rmat16": gg.config_rmat16, "grid": gg.config_grid4096,
                 "rmat18": lambda: gg.rmat(18, 16, 1)}[name]()
            yield name, False, (torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda())


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workloads", default="rmat16,grid,chunglu,hcns,batch")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    root = os.path.dirname(_HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import paper_2502_08042_amd as K

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    cache = load_cache(args.out)
    dev = device_key()
    for name, batched, t in _workloads(args.workloads.split(",")):
        t0 = time.time()
        if batched:
            vptr, off, adj = t
            cls = workload_class(off, batched=True)
            best, best_ms, ref_ms, trials = tune_batched(vptr, off, adj, reps=args.reps + 2, log=log)
        else:
            off, adj = t
            cls = workload_class(off)
            best, best_ms, ref_ms, trials = tune_single(off, adj, reps=args.reps, log=log)
        cache.setdefault(dev, {})[cls] = {
            "options": best, "ms": round(best_ms, 4), "default_ms": round(ref_ms, 4),
            "tuned_on": name, "n": int(off.numel() - 1), "m": int(adj.numel()),
            "trials": len(trials), "when": time.strftime("%Y-%m-%d %H:%M:%S")}
        log(f"[tune] {name} ({cls}): {best} {best_ms:.3f} ms (default {ref_ms:.3f} ms), "
            f"{len(trials)} trials in {time.time() - t0:.0f} s")
        del t
        torch.cuda.synchronize()
        K.release_workspaces()
        torch.cuda.empty_cache()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    tmp = args.out + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, args.out)
    print(json.dumps({dev: cache[dev]}), flush=True)


if __name__ == "__main__":
    main()
