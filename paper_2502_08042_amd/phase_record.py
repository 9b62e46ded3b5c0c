"""Timeline of one single-graph decomposition from the library's debug records (needs a GPU).

    python -m paper_2502_08042_amd.phase_record [--workload chunglu|rmat16|grid] [--mode auto]
                                                [--workgroups P]

Prints, from the phase timeline that workgroup 0 of the persistent peel kernel records (start,
work done, barrier passed, kind, round k): the grid phases grouped by kind and range of k (time to
the next barrier and workgroup 0's own work), then the tail kernel's rounds (scan, chain and
collapse rounds). With ``--workgroups P`` it also reads every workgroup's record of phases
[P, P + 64) (start and end of its work, hub tiles it took from its own tile queue, vertices it
peeled from its local queues) and prints, per phase, how the workgroups' work times spread: the
barrier waits for the slowest one.

Clock: the 100 MHz constant clock (ticks / 100 = microseconds).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = {0: "scan", 1: "expand", 2: "async", 3: "residual", 4: "tail handoff", 5: "sample check"}
TRACE_ROWS = 16384        # phase timeline rows (upper half: tail rounds)
DBG_PHASES, DBG_BLOCKS = 64, 256


def _graph(name: str):
    root = os.path.dirname(_HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import graphgen as gg
    if name == "chunglu":
        import graphgen.gpu as gp
        return gp.config_chung_lu_device()
    g = {"rmat16": gg.config_rmat16, "grid": gg.config_grid4096}[name]()
    return torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def read_trace(lib) -> np.ndarray:
    lib.kcore_debug_trace.restype = ctypes.c_int
    lib.kcore_debug_trace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    tr = np.zeros((TRACE_ROWS, 8), dtype=np.uint64)
    if lib.kcore_debug_trace(_stream(), tr.ctypes.data, TRACE_ROWS) != 0:
        raise RuntimeError("kcore_debug_trace failed")
    return tr


def grid_summary(tr: np.ndarray):
    """Grid phases by (kind, k range): count, time to the barrier, workgroup 0's work."""
    g = tr[:TRACE_ROWS // 2].astype(np.int64)
    rows = [p for p in range(1, TRACE_ROWS // 2) if g[p, 0] and g[p, 3] >= g[p, 0]]
    acc = {}
    for p in rows:
        kind, k = int(g[p, 4]) & 15, int(g[p, 4]) >> 8
        kr = k // 100 * 100 if k < 1000 else k // 500 * 500
        a = acc.setdefault((kind, kr), [0, 0.0, 0.0])
        a[0] += 1
        a[1] += (g[p, 3] - g[p, 0]) / 100.0
        a[2] += (g[p, 1] - g[p, 0]) / 100.0
    span = (g[rows[-1], 3] - g[rows[0], 0]) / 100.0 if rows else 0.0
    return acc, len(rows), span


def tail_summary(tr: np.ndarray):
    t = tr[TRACE_ROWS // 2:].astype(np.int64)
    nr = int((t[:, 0] != 0).sum())
    if nr == 0:
        return None
    t = t[:nr]
    scan = (t[:, 1] - t[:, 0]) / 100.0
    chain = (t[:, 2] - t[:, 1]) / 100.0
    peeled = np.diff(np.concatenate([[0], t[:, 6]]))
    big = np.argsort(-chain)[:3]
    return {"rounds": nr, "k_first": int(t[0, 4]), "k_last": int(t[-1, 4]),
            "total_us": round(float(scan.sum() + chain.sum()), 1),
            "scan_us": round(float(scan.sum()), 1), "scan_median_us": round(float(np.median(scan)), 2),
            "chain_us": round(float(chain.sum()), 1), "chain_median_us": round(float(np.median(chain)), 2),
            "median_peeled_per_round": int(np.median(peeled)),
            "longest_rounds": [{"k": int(t[i, 4]), "peeled": int(peeled[i]), "us": round(float(chain[i]), 1)}
                               for i in big]}


def workgroup_summary(lib, tr: np.ndarray, p0: int):
    lib.kcore_debug_blocks.restype = ctypes.c_int
    lib.kcore_debug_blocks.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    d = np.zeros((DBG_PHASES, DBG_BLOCKS, 4), dtype=np.uint64)
    if lib.kcore_debug_blocks(_stream(), d.ctypes.data) != 0:
        raise RuntimeError("kcore_debug_blocks failed")
    out = []
    for i in range(DBG_PHASES):
        s0 = d[i, :, 0].astype(np.int64)
        used = s0 > 0
        if not used.any():
            continue
        p = p0 + i
        t0 = s0[used].min()
        work = (d[i, used, 1].astype(np.int64) - t0) / 100.0
        slow = int(np.argmax(work))
        out.append({"phase": p, "kind": KINDS.get(int(tr[p, 4]) & 15, "?"), "k": int(tr[p, 4]) >> 8,
                    "barrier_us": round((int(tr[p, 3]) - int(t0)) / 100.0, 1),
                    "work_median_us": round(float(np.median(work)), 1),
                    "work_p90_us": round(float(np.percentile(work, 90)), 1),
                    "work_max_us": round(float(work.max()), 1),
                    "tiles_own_queue_mean": round(float(d[i, used, 2].mean()), 1),
                    "tiles_own_queue_slowest": int(d[i, used, 2][slow])})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="chunglu", choices=["chunglu", "rmat16", "grid"])
    ap.add_argument("--mode", default="auto")
    ap.add_argument("--workgroups", type=int, default=0, help="first phase of the per-workgroup record")
    args = ap.parse_args(argv)
    import torch
    import paper_2502_08042_amd as K
    off, adj = _graph(args.workload)
    torch.cuda.synchronize()
    out = torch.empty(off.numel() - 1, dtype=torch.int32, device=off.device)
    K.decompose(off, adj, out, mode=args.mode)  # warm-up (workspace allocation)
    extra = {"debug_phase": args.workgroups} if args.workgroups > 0 else {}
    _, st = K.decompose(off, adj, out, mode=args.mode, stats=True, **extra)
    print(f"workload {args.workload} mode {args.mode}: {st['ms']:.2f} ms, {st['rounds']} rounds, "
          f"{st['barriers']} grid barriers, {st['tail_vertices']} vertices to the tail", flush=True)
    tr = read_trace(K.lib())
    acc, nph, span = grid_summary(tr)
    print(f"\ngrid: {nph} phases in {span / 1000:.2f} ms (workgroup 0's timeline)")
    print("| kind | k from | phases | to barrier, us | workgroup 0 work, us | per phase, us |")
    print("|---|---|---|---|---|---|")
    for (kind, kr), (c, tot, wk) in sorted(acc.items(), key=lambda x: (x[0][1], x[0][0])):
        print(f"| {KINDS.get(kind, kind)} | {kr} | {c} | {tot:.0f} | {wk:.0f} | {tot / c:.1f} |")
    ts = tail_summary(tr)
    if ts:
        print("\ntail:", json.dumps(ts))
    if args.workgroups > 0:
        print(f"\nper-workgroup record of phases {args.workgroups}..{args.workgroups + DBG_PHASES - 1}:")
        print("| phase | kind | k | barrier at, us | work median | p90 | max | own-queue tiles mean | slowest's |")
        print("|---|---|---|---|---|---|---|---|---|")
        for r in workgroup_summary(K.lib(), tr, args.workgroups):
            print(f"| {r['phase']} | {r['kind']} | {r['k']} | {r['barrier_us']} | {r['work_median_us']} | "
                  f"{r['work_p90_us']} | {r['work_max_us']} | {r['tiles_own_queue_mean']} | "
                  f"{r['tiles_own_queue_slowest']} |")


if __name__ == "__main__":
    main()
