"""Summaries of rocprofv3 CSV output for the profiles kept with the library.

  python -m paper_1307_4354_amd.prof_summary trace KERNEL_TRACE_CSV --cmd "..." [--top N]
      Markdown table of kernel dispatches grouped by (kernel, grid size): count, average
      and total duration, share of the GPU time.

  python -m paper_1307_4354_amd.prof_summary traffic --fetch CSV --write CSV --kernel SUBSTR
      --grid G --copy-bytes B --cmd "..." [--sources FILE ...]
      JSON: median FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the dispatches of one
      kernel at one grid size, calibrated by the same counters on the largest plain copy
      dispatch of the run (B bytes read and B bytes written), and the SHA-256 of the
      kernel's source files, so a reader can tell whether the counters are stale.

  python -m paper_1307_4354_amd.prof_summary rates KERNEL_TRACE_CSV --fetch CSV --write CSV
      --copy-bytes B --cmd "..." [--top N]
      Markdown table per (kernel, grid size) of the trace's average duration beside the
      copy-calibrated FETCH_SIZE + WRITE_SIZE per dispatch (medians) of the counter runs, and
      the HBM rate they give; the kernels are ranked by their total traced time.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import statistics
import sys
from typing import Dict, List

HERE = os.path.dirname(os.path.abspath(__file__))
EXT_SOURCES = ["csrc/kernels.hip", "csrc/kernels_dev.h", "csrc/kernels.h"]


def sources_sha256(rel_paths: List[str]) -> str:
    h = hashlib.sha256()
    for rel in rel_paths:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(rel.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _short(name: str, width: int = 90) -> str:
    name = name.replace("cpm::(anonymous namespace)::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def trace_table(path: str, cmd: str, top: int) -> str:
    rows = list(csv.DictReader(open(path)))
    agg: Dict[tuple, List[int]] = collections.defaultdict(list)
    for r in rows:
        agg[(r["Kernel_Name"], int(r["Grid_Size_X"]))].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in agg.values())
    out = ["Command: `%s`" % cmd, "",
           "%d dispatches, %.3f ms of kernel time.  Grouped by kernel and grid size (work-items)." %
           (len(rows), total / 1e6), "",
           "| share | calls | avg us | total us | grid | kernel |", "|---:|---:|---:|---:|---:|---|"]
    for (name, grid), v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append("| %.1f%% | %d | %.2f | %.1f | %d | `%s` |" % (100.0 * sum(v) / total, len(v), sum(v) / len(v) / 1e3,
                                                             sum(v) / 1e3, grid, _short(name)))
    return "\n".join(out) + "\n"


def _counter(path: str, counter: str):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    if not rows:
        raise SystemExit("no %s rows in %s" % (counter, path))
    return rows


def _median_kib(rows, kernel: str, grid: int):
    vals = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"] and int(r["Grid_Size"]) == grid]
    if not vals:
        raise SystemExit("no dispatch of %r with grid %d" % (kernel, grid))
    return statistics.median(vals), len(vals)


def _copy_kib(rows) -> float:
    vals = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower()]
    if not vals:
        raise SystemExit("no copy dispatch to calibrate against")
    return max(vals)


def traffic(args) -> dict:
    fr = _counter(args.fetch, "FETCH_SIZE")
    wr = _counter(args.write, "WRITE_SIZE")
    f_kib, nf = _median_kib(fr, args.kernel, args.grid)
    w_kib, nw = _median_kib(wr, args.kernel, args.grid)
    cf, cw = _copy_kib(fr), _copy_kib(wr)
    kf = args.copy_bytes / (cf * 1024.0)
    kw = args.copy_bytes / (cw * 1024.0)
    fetch_b = f_kib * 1024.0 * kf
    write_b = w_kib * 1024.0 * kw
    return {"command": args.cmd, "kernel": args.kernel, "grid": args.grid, "dispatches": [nf, nw],
            "fetch_kib_median": f_kib, "write_kib_median": w_kib,
            "copy_calibration": {"bytes": args.copy_bytes, "fetch_kib": cf, "write_kib": cw,
                                 "fetch_factor": kf, "write_factor": kw},
            "fetch_bytes": fetch_b, "write_bytes": write_b, "traffic_bytes": fetch_b + write_b,
            "sources": args.sources, "source_sha256": sources_sha256(args.sources)}


def rates_table(args) -> str:
    rows = list(csv.DictReader(open(args.csv)))
    dur: Dict[tuple, List[int]] = collections.defaultdict(list)
    for r in rows:
        dur[(r["Kernel_Name"], int(r["Grid_Size_X"]))].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    fr = _counter(args.fetch, "FETCH_SIZE")
    wr = _counter(args.write, "WRITE_SIZE")
    kf = args.copy_bytes / (_copy_kib(fr) * 1024.0)
    kw = args.copy_bytes / (_copy_kib(wr) * 1024.0)
    fk: Dict[tuple, List[float]] = collections.defaultdict(list)
    wk: Dict[tuple, List[float]] = collections.defaultdict(list)
    for src, dst in ((fr, fk), (wr, wk)):
        for r in src:
            dst[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    total = sum(sum(v) for v in dur.values())
    out = ["Command: `%s`" % args.cmd, "",
           "Durations from the kernel trace; traffic = median FETCH_SIZE x %.3f + median WRITE_SIZE x %.3f "
           "per dispatch (factors from a plain copy of %.0f bytes in the counter runs); rate = traffic / "
           "average duration.  Kernels with no counter dispatch at that grid size are left out." %
           (kf, kw, args.copy_bytes), "",
           "| share of traced time | calls | avg us | fetch MB | write MB | GB/s | grid | kernel |",
           "|---:|---:|---:|---:|---:|---:|---:|---|"]
    shown = 0
    for key, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        if key not in fk or key not in wk:
            continue
        avg_ns = sum(v) / len(v)
        fb = statistics.median(fk[key]) * 1024.0 * kf
        wb = statistics.median(wk[key]) * 1024.0 * kw
        out.append("| %.1f%% | %d | %.2f | %.1f | %.1f | %.0f | %d | `%s` |" % (
            100.0 * sum(v) / total, len(v), avg_ns / 1e3, fb / 1e6, wb / 1e6, (fb + wb) / avg_ns, key[1],
            _short(key[0])))
        shown += 1
        if shown >= args.top:
            break
    return "\n".join(out) + "\n"


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--cmd", required=True)
    t.add_argument("--top", type=int, default=30)
    q = sub.add_parser("traffic")
    q.add_argument("--fetch", required=True)
    q.add_argument("--write", required=True)
    q.add_argument("--kernel", required=True)
    q.add_argument("--grid", type=int, required=True)
    q.add_argument("--copy-bytes", type=float, required=True)
    q.add_argument("--cmd", required=True)
    q.add_argument("--sources", nargs="*", default=EXT_SOURCES)
    rt = sub.add_parser("rates")
    rt.add_argument("csv")
    rt.add_argument("--fetch", required=True)
    rt.add_argument("--write", required=True)
    rt.add_argument("--copy-bytes", type=float, required=True)
    rt.add_argument("--cmd", required=True)
    rt.add_argument("--top", type=int, default=25)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        sys.stdout.write(trace_table(a.csv, a.cmd, a.top))
    elif a.mode == "rates":
        sys.stdout.write(rates_table(a))
    else:
        json.dump(traffic(a), sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()
