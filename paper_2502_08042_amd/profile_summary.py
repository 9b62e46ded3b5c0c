"""Summaries of rocprofv3 output for profiles/ (runs on the host after the profiled runs).

    python -m paper_2502_08042_amd.profile_summary stats DIR [--match peel_kernel,tail_kernel]
        per-kernel calls / total / average / min / max from a --kernel-trace --stats run
    python -m paper_2502_08042_amd.profile_summary traffic --workload W --mode M
        --copy-fetch DIR --copy-write DIR --fetch DIR --write DIR --match peel_kernel,tail_kernel
        HBM bytes per launch from FETCH_SIZE / WRITE_SIZE runs, each scaled by what the same counter
        reads for a plain device copy of known size (bench.py --copy-calibration); prints the JSON
        that bench.py reads back (keyed by the kernel source hash)
    python -m paper_2502_08042_amd.profile_summary counters DIR --match peel_kernel
        mean per dispatch of every counter in a --pmc run
    python -m paper_2502_08042_amd.profile_summary dispatches DIR --match batched_kernel --first 5
        durations of the first N dispatches of a kernel, in launch order, from a --kernel-trace run

DIR is the rocprofv3 output directory (-d); its CSV files are found recursively.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    for fn in files:
        with open(fn, newline="") as f:
            yield from csv.DictReader(f)


def _col(row: dict, *names):
    for n in names:
        if n in row:
            return row[n]
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def kernel_stats(d: str, match):
    out = []
    for r in _rows(d, "kernel_stats.csv"):
        name = _col(r, "Name", "KernelName", "Kernel_Name")
        if match and not any(m in name for m in match):
            continue
        out.append({"kernel": _short(name), "calls": int(_col(r, "Calls")),
                    "total_ms": float(_col(r, "TotalDurationNs")) / 1e6,
                    "avg_ms": float(_col(r, "AverageNs")) / 1e6,
                    "min_ms": float(_col(r, "MinNs")) / 1e6, "max_ms": float(_col(r, "MaxNs")) / 1e6})
    return out


def counter_means(d: str, match, counter=None, first: int = 0):
    """Mean per dispatch of each counter, per kernel (dispatches summed over counter instances);
    with `first`, over each kernel's first dispatches in launch order only."""
    per = defaultdict(lambda: defaultdict(float))  # (kernel, dispatch) -> counter -> value
    for r in _rows(d, "counter_collection.csv"):
        name = _col(r, "Kernel_Name", "Kernel-Name", "KernelName")
        if match and not any(m in name for m in match):
            continue
        cname = _col(r, "Counter_Name", "Counter-Name", "CounterName")
        if counter and cname != counter:
            continue
        disp = _col(r, "Dispatch_Id", "Dispatch-Id", "DispatchId")
        per[(_short(name), disp)][cname] += float(_col(r, "Counter_Value", "Counter-Value", "CounterValue"))
    acc = defaultdict(lambda: defaultdict(list))
    seen = defaultdict(int)
    for (k, _), cs in sorted(per.items(), key=lambda kv: (kv[0][0], int(kv[0][1]))):
        seen[k] += 1
        if first and seen[k] > first:
            continue
        for c, v in cs.items():
            acc[k][c].append(v)
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--match", default="")
    b = sub.add_parser("traffic")
    for k in ("copy-fetch", "copy-write", "fetch", "write"):
        b.add_argument("--" + k, required=True)
    b.add_argument("--match", required=True)
    b.add_argument("--workload", required=True)
    b.add_argument("--mode", default="auto")
    b.add_argument("--first", type=int, default=0, help="only each kernel's first N dispatches")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--match", default="")
    e = sub.add_parser("dispatches")
    e.add_argument("dir")
    e.add_argument("--match", required=True)
    e.add_argument("--first", type=int, default=0)
    args = ap.parse_args(argv)
    match = [m for m in args.match.split(",") if m]
    if args.cmd == "stats":
        rows = kernel_stats(args.dir, match)
        print("| kernel | calls | total ms | avg ms | min ms | max ms |")
        print("|---|---|---|---|---|---|")
        for r in rows:
            print(f"| `{r['kernel']}` | {r['calls']} | {r['total_ms']:.3f} | {r['avg_ms']:.3f} | "
                  f"{r['min_ms']:.3f} | {r['max_ms']:.3f} |")
        print(f"\nsum of averages: {sum(r['avg_ms'] for r in rows):.3f} ms")
        return
    if args.cmd == "counters":
        print(json.dumps(counter_means(args.dir, match), indent=1, sort_keys=True))
        return
    if args.cmd == "dispatches":
        rows = [r for r in _rows(args.dir, "kernel_trace.csv")
                if any(m in _col(r, "Kernel_Name", "KernelName") for m in match)]
        rows.sort(key=lambda r: int(_col(r, "Start_Timestamp")))
        ms = [(int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e6 for r in rows]
        if args.first > 0:
            ms = ms[:args.first]
        print(json.dumps({"dispatches": len(ms), "mean_ms": round(sum(ms) / max(len(ms), 1), 4),
                          "min_ms": round(min(ms), 4) if ms else None,
                          "max_ms": round(max(ms), 4) if ms else None, "each_ms": [round(x, 4) for x in ms]}))
        return
    copy = ["copyBuffer", "copy_kernel", "elementwise", "Copy"]
    cf = counter_means(args.copy_fetch, copy, "FETCH_SIZE")
    cw = counter_means(args.copy_write, copy, "WRITE_SIZE")
    cfk = max(v["FETCH_SIZE"] for v in cf.values())
    cwk = max(v["WRITE_SIZE"] for v in cw.values())
    copy_bytes = 1 << 30
    ff, wf = copy_bytes / (cfk * 1024), copy_bytes / (cwk * 1024)
    fk = {k: v["FETCH_SIZE"] for k, v in counter_means(args.fetch, match, "FETCH_SIZE", args.first).items()}
    wk = {k: v["WRITE_SIZE"] for k, v in counter_means(args.write, match, "WRITE_SIZE", args.first).items()}
    sys.path.insert(0, ROOT)
    import bench
    fb = sum(fk.values()) * 1024 * ff
    wb = sum(wk.values()) * 1024 * wf
    print(json.dumps({
        "kernels": sorted(fk), "workload": args.workload, "mode": args.mode,
        "kernel_source_sha": bench.kernel_sha(),
        "fetch_size_kib_per_launch": fk, "write_size_kib_per_launch": wk,
        "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes, "fetch_size_kib": cfk,
                             "write_size_kib": cwk, "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
        "fetch_bytes_per_launch": int(fb), "write_bytes_per_launch": int(wb),
        "bytes_per_launch": int(fb + wb)}, indent=1))


if __name__ == "__main__":
    main()
