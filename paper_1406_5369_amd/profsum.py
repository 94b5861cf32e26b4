"""Summaries of rocprofv3 kernel traces, per kernel and launch shape.

    python -m paper_1406_5369_amd.profsum RESULTS.db [--top N] [--match SUBSTR]
    python -m paper_1406_5369_amd.profsum kernel_trace.csv

Reads a rocprofv3 ``--kernel-trace`` result (the SQLite ``*_results.db`` that
rocprofv3 writes by default, or a ``kernel_trace.csv``) and prints, for each
(kernel, grid) pair, the number of dispatches and their total / average
duration, so that launches of one kernel on different grid levels are told
apart.  It reads only rocprofv3's output files.
"""

from __future__ import annotations

import argparse
import csv
import re
import sqlite3
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    name = name.strip().replace("(anonymous namespace)::", "")
    name = re.sub(r"\([^()]*\)$", "", name)
    return name.replace("void ", "")


def load(path: str):
    rows = []
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        cur = con.cursor()
        q = "select name, duration, grid_x, grid_y, grid_z, workgroup_x from kernels"
        for name, dur, gx, gy, gz, wx in cur.execute(q):
            rows.append((short_name(name), float(dur), int(gx), int(gy), int(gz), int(wx)))
    else:
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                dur = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
                rows.append((short_name(r["Kernel_Name"]), dur, int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]),
                             int(r["Grid_Size_Z"]), int(r["Workgroup_Size_X"])))
    return rows


def summarize(rows, match: str | None = None):
    agg = defaultdict(lambda: [0, 0.0])
    for name, dur, gx, gy, gz, wx in rows:
        if match and match not in name:
            continue
        key = (name, gx // max(wx, 1), gy, gz)
        agg[key][0] += 1
        agg[key][1] += dur
    total = sum(v[1] for v in agg.values())
    out = []
    for (name, bx, gy, gz), (cnt, tot) in agg.items():
        out.append(dict(kernel=name, blocks_x=bx, grid_y=gy, grid_z=gz, calls=cnt, total_ms=tot / 1e6,
                        avg_us=tot / cnt / 1e3, pct=100.0 * tot / total if total else 0.0))
    out.sort(key=lambda d: -d["total_ms"])
    return out


def counters(path: str, match: str | None = None):
    """Average value per dispatch of every collected counter, per (kernel, blocks)."""
    con = sqlite3.connect(path)
    q = ("select kernel_name, grid_size_x, workgroup_size_x, counter_name, value from counters_collection")
    agg = defaultdict(lambda: [0, 0.0])
    for name, gx, wx, cname, val in con.execute(q):
        k = short_name(name)
        if match and match not in k:
            continue
        key = (k, int(gx) // max(int(wx), 1), cname)
        agg[key][0] += 1
        agg[key][1] += float(val)
    out = []
    for (k, bx, cname), (cnt, tot) in agg.items():
        out.append(dict(kernel=k, blocks_x=bx, counter=cname, dispatches=cnt, avg=tot / cnt))
    out.sort(key=lambda d: (d["kernel"], d["blocks_x"], d["counter"]))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--match", default=None)
    ap.add_argument("--counters", action="store_true", help="per-dispatch counter averages (--pmc runs)")
    a = ap.parse_args(argv)
    if a.counters:
        print(f"{'counter':>12} {'avg/dispatch':>16} {'n':>5} {'blocks':>7}  kernel")
        for d in counters(a.trace, a.match):
            print(f"{d['counter']:>12} {d['avg']:16.1f} {d['dispatches']:5d} {d['blocks_x']:7d}  {d['kernel']}")
        return 0
    res = summarize(load(a.trace), a.match)
    print(f"{'pct':>6} {'total_ms':>10} {'calls':>6} {'avg_us':>10} {'blocks':>7} {'gy':>4}  kernel")
    for d in res[: a.top]:
        print(f"{d['pct']:6.2f} {d['total_ms']:10.3f} {d['calls']:6d} {d['avg_us']:10.2f} {d['blocks_x']:7d} "
              f"{d['grid_y']:4d}  {d['kernel']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
