"""Summaries of rocprofv3 kernel traces, per kernel and launch shape.

    python -m paper_1406_5369_amd.profsum RESULTS.db [--top N] [--match SUBSTR]
    python -m paper_1406_5369_amd.profsum kernel_trace.csv
    python -m paper_1406_5369_amd.profsum --counters PMC_RESULTS.db
    python -m paper_1406_5369_amd.profsum --traffic FETCH.db WRITE.db --bench BENCH.json --out traffic.json

Reads a rocprofv3 ``--kernel-trace`` result (the SQLite ``*_results.db`` that
rocprofv3 writes by default, or a ``kernel_trace.csv``) and prints, for each
(kernel, grid) pair, the number of dispatches and their total / average
duration, so that launches of one kernel on different grid levels are told
apart.  ``--counters`` prints per-dispatch averages of the counters of a
``--pmc`` run.  ``--traffic`` turns one ``FETCH_SIZE`` run and one
``WRITE_SIZE`` run of the benchmark (started with ``--calibrate-copy``, so
that each run also holds three 1 GiB device copies) into HBM bytes per launch
of the benchmark's dominant kernel: each counter is scaled by the factor that
makes it read 1 GiB for the copy kernel, and the record is tagged with the
hash of the device sources it was measured on.  It reads only rocprofv3's
output files and the benchmark's JSON line.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_BYTES = 1 << 30  # size of each calibration copy (bench.py --calibrate-copy)
BX = 64               # tile width of the sweep kernels


def kernel_source_hash() -> str:
    """Hash of the device-code sources (kernels and their shared headers)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.startswith(("mg_smooth", "mg_resid", "mg_transfer", "mg_kern", "mg_internal")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_kernel(dim: int, word: int, by: int, pd: int, var: bool = False, wv: int = 4, flags: int = 0) -> str:
    """Demangled name of an RBGS sweep with the given tile height, prefetch
    depth and wavefronts: plain (flags 0), or with flags 4 the FP64 sweep that
    also sums the residual norm of its incoming iterate."""
    t = {2: "_Float16", 4: "float", 8: "double"}[word]
    v = "true" if var else "false"
    if dim == 2:
        return f"mg::k_smooth2d<{t}, 0, {v}, {by}, {flags}>"
    if wv == 1:  # one wavefront per tile, rows in registers
        return f"mg::k_smooth3d_rc<{t}, 0, {v}, {by}, {pd}, {flags}>"
    return f"mg::k_smooth3d<{t}, 0, {v}, {by}, {pd}, {flags}, {wv}>"


def pass_kernel(dim: int, by: int, pd: int, var: bool = False, ir: bool = True, wv: int = 4, pairs: int = 0,
                word: int = 4) -> str:
    """Demangled name of the finest-level FP64 refinement pass (updating, as
    in a refinement step) or FP64 norm pass with the given tile height,
    prefetch depth and wavefronts (pairs: the variant with two nodes per lane,
    whose correction / residual words are float, or binary16 with word 2)."""
    v = "true" if var else "false"
    e = "_Float16" if word == 2 else "float"
    if pairs and dim == 3:
        return f"mg::k_ir3d_p<{by}, {pd}, 0, {wv}, {e}>" if ir else f"mg::k_norm3d_p<{by}, {pd}, {wv}>"
    if pairs:
        return f"mg::k_ir2d_p<{pd}, 0, {e}>" if ir else f"mg::k_norm2d_p<{pd}>"
    if ir:
        return f"mg::k_ir2d<{v}, {by}, 0>" if dim == 2 else f"mg::k_ir3d<{v}, {by}, {pd}, 0, {wv}>"
    return f"mg::k_norm2d<{v}, {by}>" if dim == 2 else f"mg::k_norm3d<{v}, {by}, {pd}, {wv}>"


def pass_blocks(dim: int, n: int, by: int, zchunk: int, pairs: int = 0) -> int:
    """Workgroups of a refinement / norm pass: tiles of (BX - 2) x (by - 2)
    inner points (a one-point halo; 2 BX wide with two nodes per lane, whose
    x-neighbours outside the tile are loaded on their own), times z-chunks in
    3D; in 2D with two nodes per lane, strips of 2 BX nodes in chunks of
    zchunk rows, four chunks per workgroup."""
    m = n - 2
    cd = lambda a, b: -(-a // b)  # noqa: E731
    if pairs and dim == 2:  # four wavefronts per workgroup, each marching zchunk rows
        return cd(m, 2 * BX) * cd(cd(m, zchunk), 4)
    b = cd(m, 2 * BX if pairs else BX - 2) * cd(m, by - 2)
    return b if dim == 2 else b * cd(m, zchunk)


def sweep_blocks(dim: int, n: int, by: int, zchunk: int) -> int:
    """Workgroups of one RBGS sweep over an n^dim node grid: tiles of
    (BX - 4) x (by - 4) inner points (a two-point halo), times z-chunks in 3D."""
    m = n - 2
    cd = lambda a, b: -(-a // b)  # noqa: E731
    b = cd(m, BX - 4) * cd(m, by - 4)
    return b if dim == 2 else b * cd(m, zchunk)


def short_name(name: str) -> str:
    name = name.strip().replace("(anonymous namespace)::", "")
    name = re.sub(r"\([^()]*\)$", "", name)
    return name.replace("void ", "")


def load(path: str, from_kernel: str | None = None):
    """Dispatches in start order; with from_kernel, only those from the first
    dispatch whose name contains it (e.g. the first solve after setup)."""
    rows = []
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        cur = con.cursor()
        q = "select name, duration, grid_x, grid_y, grid_z, workgroup_x from kernels order by start"
        for name, dur, gx, gy, gz, wx in cur.execute(q):
            rows.append((short_name(name), float(dur), int(gx), int(gy), int(gz), int(wx)))
    else:
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                dur = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
                rows.append((short_name(r["Kernel_Name"]), dur, int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]),
                             int(r["Grid_Size_Z"]), int(r["Workgroup_Size_X"])))
    if from_kernel:
        first = next((i for i, r in enumerate(rows) if from_kernel in r[0]), len(rows))
        rows = rows[first:]
    return rows


IDLE_FRAC = 0.25  # a dispatch under this fraction of its kernel's median did no work


def summarize(rows, match: str | None = None):
    """Per (kernel, grid): dispatches, total and average time.  Dispatches
    shorter than IDLE_FRAC of the median of their kernel and grid are counted
    apart as idle: launches of a step queued after the solve finished, whose
    workgroups all exit at the stop flag; they stay in the totals."""
    agg = defaultdict(list)
    for name, dur, gx, gy, gz, wx in rows:
        if match and match not in name:
            continue
        agg[(name, gx // max(wx, 1), gy, gz)].append(dur)
    total = sum(sum(v) for v in agg.values())
    out = []
    for (name, bx, gy, gz), durs in agg.items():
        med = sorted(durs)[len(durs) // 2]
        work = [d for d in durs if d >= IDLE_FRAC * med]
        tot = sum(durs)
        out.append(dict(kernel=name, blocks_x=bx, grid_y=gy, grid_z=gz, calls=len(work), idle=len(durs) - len(work),
                        total_ms=tot / 1e6, avg_us=sum(work) / len(work) / 1e3,
                        pct=100.0 * tot / total if total else 0.0))
    out.sort(key=lambda d: -d["total_ms"])
    return out


def counters(path: str, match: str | None = None):
    """Average value per dispatch of every collected counter, per (kernel,
    blocks), over the dispatches that read at least IDLE_FRAC of the largest
    reading (the others, stop-flag exits, are counted as idle)."""
    con = sqlite3.connect(path)
    q = ("select kernel_name, grid_size_x, workgroup_size_x, counter_name, value from counters_collection")
    agg = defaultdict(list)
    for name, gx, wx, cname, val in con.execute(q):
        k = short_name(name)
        if match and match not in k:
            continue
        agg[(k, int(gx) // max(int(wx), 1), cname)].append(float(val))
    out = []
    for (k, bx, cname), vals in agg.items():
        keep = [v for v in vals if v >= IDLE_FRAC * max(vals)] or vals
        out.append(dict(kernel=k, blocks_x=bx, counter=cname, dispatches=len(keep), idle=len(vals) - len(keep),
                        avg=sum(keep) / len(keep)))
    out.sort(key=lambda d: (d["kernel"], d["blocks_x"], d["counter"]))
    return out


def _counter_rows(path: str, cname: str):
    con = sqlite3.connect(path)
    q = ("select kernel_name, grid_size_x, workgroup_size_x, value from counters_collection "
         "where counter_name = ?")
    per = defaultdict(list)
    for name, gx, wx, val in con.execute(q, (cname,)):
        per[(short_name(name), int(gx) // max(int(wx), 1))].append(float(val))
    return per


def _bench_line(path: str) -> dict:
    with open(path) as fh:
        lines = [ln for ln in fh if ln.lstrip().startswith("{")]
    if not lines:
        raise SystemExit(f"{path}: no JSON line")
    return json.loads(lines[-1])


def _entry(runs, kname: str, blocks: int, algo: float) -> dict | None:
    """Calibrated bytes per launch of one kernel and grid in both counter runs;
    dispatches under IDLE_FRAC of the largest reading of their counter (stop
    flag set, no work) are left out."""
    ent = {"kernel": kname, "blocks": blocks}
    total = 0.0
    for cname, (per, calib_kib, factor) in runs.items():
        vals = per.get((kname, blocks))
        if not vals:
            return None
        keep = [v for v in vals if v >= IDLE_FRAC * max(vals)]
        avg = sum(keep) / len(keep)
        ent[cname] = {"kib_per_dispatch": avg, "dispatches": len(keep), "idle": len(vals) - len(keep),
                      "factor": factor}
        total += avg * 1024.0 * factor
    ent["bytes_per_launch"] = total
    ent["ratio_to_algorithmic"] = total / algo
    return ent


def traffic(fetch_db: str, write_db: str, bench_json: str) -> dict:
    """HBM bytes per launch of the benchmark's finest-level sweep and
    refinement pass, from one FETCH_SIZE and one WRITE_SIZE run (KiB per
    dispatch), each calibrated on the 1 GiB copies of the same run.  The tile
    autotuner launches every candidate geometry on the finest level during
    setup, so the record holds one entry per geometry present in both runs,
    keyed "by,zchunk,prefetch,waves"."""
    b = _bench_line(bench_json)
    cfg = b["config"]
    dim, n = cfg["dim"], cfg["n"]
    word = 4 if "f32" in b["dtype"] else 8
    var = "varcoef" in cfg["workload"]
    algo = (4 if var else 3) * word * (n - 2) ** dim
    runs = {}
    for db, cname in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        per = _counter_rows(db, cname)
        copies = [v for (k, _), vals in per.items() if k == "mg::k_copy_bytes" for v in vals]
        if not copies:
            raise SystemExit(f"{db}: no k_copy_bytes dispatches (run the benchmark with --calibrate-copy)")
        calib_kib = max(copies)
        runs[cname] = (per, calib_kib, COPY_BYTES / (calib_kib * 1024.0))
    zcs = (4, 8, 16, 32, 64, 128, 256) if dim == 3 else (1,)
    pds = (1, 2) if dim == 3 else (1,)
    configs = {}
    for by, wv in ((8, 4), (16, 4), (32, 4), (16, 8), (32, 8), (8, 1), (12, 1)):
        if dim == 2 and wv != 4:
            continue
        for pd in pds:
            for zc in zcs:
                ent = _entry(runs, sweep_kernel(dim, word, by, pd, var, wv), sweep_blocks(dim, n, by, zc), algo)
                if ent:
                    configs[f"{by},{zc},{pd},{wv}"] = ent
    if not configs:
        raise SystemExit("no finest-level sweep dispatches found in both runs")
    # refinement pass (mixed precision): FP64 u and f read, FP32 e read, FP64 u and FP32 r written
    ir = word == 4
    algo_pass = ((32 if ir else 16) + (8 if var else 0)) * (n - 2) ** dim
    pass_configs = {}
    for by, wv in ((8, 4), (16, 4), (32, 4), (16, 8), (32, 8)):
        if dim == 2 and wv != 4:
            continue
        for pd in pds:
            for zc in zcs:
                for pr in ((0, 1) if dim == 3 and not var else (0,)):
                    ent = _entry(runs, pass_kernel(dim, by, pd, var, ir, wv, pr), pass_blocks(dim, n, by, zc, pr),
                                 algo_pass)
                    if ent:
                        pass_configs[f"{by},{zc},{pd},{wv}" + (",p" if pr else "")] = ent
    by, zc, pd, wv = b["extra"]["fine_tiles"]["smooth"][:4]
    pby, pzc, ppd, pwv = b["extra"]["fine_tiles"]["norm_or_refinement"][:4]
    ppr = b["extra"]["fine_tiles"]["norm_or_refinement"][5] if len(b["extra"]["fine_tiles"]["norm_or_refinement"]) > 5 else 0
    return {
        "workload": cfg["workload"],
        "source_hash": kernel_source_hash(),
        "algorithmic_bytes": algo,
        "algorithmic_bytes_pass": algo_pass,
        "calibration": {c: {"copy_kib_per_GiB": v[1], "factor": v[2]} for c, v in runs.items()},
        "bench_tiles": f"{by},{zc},{pd},{wv}",
        "bench_pass_tiles": f"{pby},{pzc},{ppd},{pwv}" + (",p" if ppr else ""),
        "configs": configs,
        "pass_configs": pass_configs,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("trace", nargs="+")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--match", default=None)
    ap.add_argument("--from-kernel", default=None, help="skip dispatches before the first one of this kernel")
    ap.add_argument("--counters", action="store_true", help="per-dispatch counter averages (--pmc runs)")
    ap.add_argument("--traffic", action="store_true", help="FETCH.db WRITE.db -> bytes per launch")
    ap.add_argument("--bench", help="benchmark output (JSON line) of the counter runs")
    ap.add_argument("--out", help="traffic JSON to update (one record per workload)")
    a = ap.parse_args(argv)
    if a.traffic:
        if len(a.trace) != 2 or not a.bench:
            ap.error("--traffic needs FETCH.db WRITE.db and --bench")
        rec = traffic(a.trace[0], a.trace[1], a.bench)
        print(json.dumps(rec, indent=1))
        if a.out:
            allrec = {}
            if os.path.exists(a.out):
                with open(a.out) as fh:
                    allrec = json.load(fh)
            allrec[rec["workload"]] = rec
            with open(a.out, "w") as fh:
                json.dump(allrec, fh, indent=1, sort_keys=True)
                fh.write("\n")
        return 0
    a.trace = a.trace[0]
    if a.counters:
        print(f"{'counter':>12} {'avg/dispatch':>16} {'n':>5} {'idle':>5} {'blocks':>7}  kernel")
        for d in counters(a.trace, a.match):
            print(f"{d['counter']:>12} {d['avg']:16.1f} {d['dispatches']:5d} {d['idle']:5d} {d['blocks_x']:7d}  "
                  f"{d['kernel']}")
        return 0
    res = summarize(load(a.trace, a.from_kernel), a.match)
    print(f"{'pct':>6} {'total_ms':>10} {'calls':>6} {'idle':>5} {'avg_us':>10} {'blocks':>7} {'gy':>4}  kernel")
    for d in res[: a.top]:
        print(f"{d['pct']:6.2f} {d['total_ms']:10.3f} {d['calls']:6d} {d['idle']:5d} {d['avg_us']:10.2f} "
              f"{d['blocks_x']:7d} {d['grid_y']:4d}  {d['kernel']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
