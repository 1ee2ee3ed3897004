"""Summaries of rocprofv3 runs of this library's kernels (kernel trace, counter passes).

    python -m paper_2512_02577_amd.rocprof_summary trace DIR [--top K]
        per-kernel totals and averages from a --kernel-trace run (CSV output under DIR)
    python -m paper_2512_02577_amd.rocprof_summary traffic --trace DIR --fetch DIR --write DIR
                                                          --kernel REGEX --name NAME [--grid G ...]
                                                          [--bytes B] [--record] [--summary PATH]
        average duration and HBM traffic per dispatch of the matching kernel (grouped by grid
        size, the groups listed by --grid), FETCH_SIZE and WRITE_SIZE scaled by what the same
        counters read for the largest plain device copy in the run (a blit of known size:
        FETCH should read its size, WRITE its size); --record also writes
        profiles/NAME.traffic.json with the SHA-256 of the kernel sources.

Reads CSV files only; prints markdown.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2512_02577_amd/csrc/bodies.h", "paper_2512_02577_amd/csrc/sumfac.h",
                  "paper_2512_02577_amd/csrc/kernels_impl.h", "paper_2512_02577_amd/csrc/dispatch.h",
                  "paper_2512_02577_amd/csrc/constants.h", "paper_2512_02577_amd/csrc/launch.h",
                  "paper_2512_02577_amd/csrc/march.h",
                  "paper_2512_02577_amd/csrc/kernels_3d_f64.hip"]
COPY_KERNEL = re.compile(r"copyBuffer|copy_kernel|CopyKernel", re.I)


def _source(rel: str, rev: str | None) -> bytes:
    """A kernel source as built for the profiled run: the working tree, or a git revision."""
    if not rev:
        return open(os.path.join(ROOT, rel), "rb").read()
    import subprocess

    return subprocess.run(["git", "-C", ROOT, "show", f"{rev}:{rel}"], check=True, capture_output=True).stdout


def _rows(d: str, suffix: str):
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _grid(row) -> int:
    for k in ("Grid_Size", "Grid_Size_X"):
        if k in row and row[k]:
            return int(float(row[k]))
    return 0


def _wg(row) -> int:
    for k in ("Workgroup_Size", "Workgroup_Size_X"):
        if k in row and row[k]:
            return int(float(row[k]))
    return 1


def trace_table(d: str, top: int = 25) -> str:
    rows = _rows(d, "kernel_trace.csv")
    agg = defaultdict(lambda: [0, 0.0])
    for r in rows:
        t = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3  # us
        a = agg[r["Kernel_Name"]]
        a[0] += 1
        a[1] += t
    total = sum(v[1] for v in agg.values()) or 1.0
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"| `{name[:110]}` | {c} | {t * 1e-3:.2f} | {t / c:.2f} | {100 * t / total:.1f} |")
    return "\n".join(lines)


def _durations(d: str, pattern: re.Pattern):
    """(workgroups, duration us) of every dispatch of the matching kernel."""
    out = []
    for r in _rows(d, "kernel_trace.csv"):
        if pattern.search(r["Kernel_Name"]):
            out.append((_grid(r) // max(1, _wg(r)), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3))
    return out


def _counter(d: str, counter: str):
    """[(kernel name, workgroups, value KiB)] per dispatch."""
    out = []
    for r in _rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") == counter:
            out.append((r["Kernel_Name"], _grid(r) // max(1, _wg(r)), float(r["Counter_Value"]), _grid(r)))
    return out


def _calibration(rows):
    """The largest plain device copy of the run: (threads, counter KiB)."""
    best = None
    for name, wg, kib, threads in rows:
        if COPY_KERNEL.search(name) and (best is None or kib > best[1]):
            best = (threads, kib)
    return best


def traffic(args) -> int:
    pat = re.compile(args.kernel)
    durs = _durations(args.trace, pat)
    fetch = _counter(args.fetch, "FETCH_SIZE")
    write = _counter(args.write, "WRITE_SIZE")
    cal_f, cal_w = _calibration(fetch), _calibration(write)
    copy_bytes = args.copy_bytes
    sf = copy_bytes / (cal_f[1] * 1024) if cal_f else 1.0
    sw = copy_bytes / (cal_w[1] * 1024) if cal_w else 1.0
    print(f"Calibration: the largest device copy in the run moves {copy_bytes / 2**20:.0f} MiB each way; "
          f"FETCH_SIZE read {cal_f[1] if cal_f else float('nan'):.0f} KiB (scale {sf:.4f}), "
          f"WRITE_SIZE {cal_w[1] if cal_w else float('nan'):.0f} KiB (scale {sw:.4f}).\n")
    groups = args.grid or sorted({g for g, _ in durs})
    lines = ["| workgroups | dispatches | avg us | FETCH KiB | WRITE KiB | scaled MB | algorithmic MB | ratio |",
             "|---|---|---|---|---|---|---|---|"]
    rec = None
    for g in groups:
        ds = [t for gg, t in durs if gg == g]
        fs = [k for n, gg, k, _ in fetch if pat.search(n) and gg == g]
        ws = [k for n, gg, k, _ in write if pat.search(n) and gg == g]
        if not ds:
            continue
        avg = sum(ds) / len(ds)
        f = sum(fs) / len(fs) if fs else float("nan")
        w = sum(ws) / len(ws) if ws else float("nan")
        scaled = (f * 1024 * sf + w * 1024 * sw)
        alg = args.bytes.get(g) if args.bytes else None
        lines.append(f"| {g} | {len(ds)} | {avg:.2f} | {f:.0f} | {w:.0f} | {scaled / 1e6:.2f} | "
                     f"{alg / 1e6 if alg else float('nan'):.2f} | {scaled / alg if alg else float('nan'):.3f} |")
        if rec is None or len(ds) > rec["dispatches"]:
            rec = {"workgroups": g, "dispatches": len(ds), "avg_us": avg, "fetch_bytes_per_launch": int(f * 1024 * sf),
                   "write_bytes_per_launch": int(w * 1024 * sw)}
    print("\n".join(lines))
    if args.record and rec:
        rec.update({"kernel": args.kernel, "method": f"FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two "
                    f"rocprofv3 --pmc runs, each scaled by the same counter on the largest plain device copy "
                    f"of the run ({copy_bytes} B read and written): FETCH x {sf:.4f}, WRITE x {sw:.4f}",
                    "summary": args.summary or f"profiles/{args.name}.md",
                    "sources_sha256": {rel: hashlib.sha256(_source(rel, args.git_rev)).hexdigest()
                                       for rel in KERNEL_SOURCES}})
        with open(os.path.join(ROOT, "profiles", f"{args.name}.traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--top", type=int, default=25)
    f = sub.add_parser("traffic")
    f.add_argument("--trace", required=True)
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--kernel", required=True)
    f.add_argument("--name", required=True)
    f.add_argument("--grid", type=int, nargs="*")
    f.add_argument("--bytes", type=str, default="", help="algorithmic bytes per launch by grid: g1=b1,g2=b2")
    f.add_argument("--copy-bytes", type=int, default=2 ** 30)
    f.add_argument("--record", action="store_true")
    f.add_argument("--summary", default=None, help="the profile summary the record belongs to (default profiles/NAME.md)")
    f.add_argument("--git-rev", default=None, help="hash the kernel sources of this revision (the profiled build)")
    args = ap.parse_args(argv)
    if args.cmd == "trace":
        print(trace_table(args.dir, args.top))
        return 0
    args.bytes = {int(k): int(v) for k, v in (kv.split("=") for kv in args.bytes.split(",") if kv)}
    return traffic(args)


if __name__ == "__main__":
    sys.exit(main())
