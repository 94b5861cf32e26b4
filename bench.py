#!/usr/bin/env python3
"""Benchmark of the MI355X multigrid solver.

One step = one complete solve, from u = 0 to a relative residual of 1e-8, of
the 3D Poisson problem -Laplace(u) = f on 513^3 nodes (h = 1/512, zero
Dirichlet boundary, f i.i.d. U[-1, 1] from numpy default_rng(0) with a zeroed
boundary), by FP32 V(2,2) red-black Gauss-Seidel cycles inside FP64 iterative
refinement.  Inputs are resident in HBM before the timed region.

Printed: one JSON line with fine-grid DoF/s (value), the plain FP64 solve of
the same problem for context, the roofline of the dominant kernel (of the
finest-level FP32 smoothing sweep and the FP64 refinement pass, the one with
the larger total time; both timed with HIP events on the solver's stream over
the timed region, the other reported beside it) and the CPU oracle timed on a
bounded sample.

The default line also carries, in `extra`, shorter runs of the batched form
(512 uneven 2D grids, solves/s and DoF/s beside the same grids solved one by
one in FP64) and of the serving form (saturated solves/s, p50/p99 latency per
arrival rate), and the CPU oracle on one thread and on all physical cores.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--no-forms]
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1406_5369_amd.profsum import (  # noqa: E402
    kernel_source_hash,
    pass_blocks,
    pass_kernel,
    sweep_blocks,
    sweep_kernel,
)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, datasheet

WORKLOADS = {
    # name: dim, n, precision, rhs, tol
    "poisson3d_513_fp32ir": dict(dim=3, n=513, precision=1, rhs=("uniform", 0), tol=1e-8),
    "poisson3d_513_fp64": dict(dim=3, n=513, precision=0, rhs=("uniform", 0), tol=1e-8),
    # the same problem with binary16 cycle fields (float arithmetic) in FP64 refinement
    "poisson3d_513_fp16ir": dict(dim=3, n=513, precision=2, rhs=("uniform", 0), tol=1e-8),
    "poisson2d_129_sine_fp64": dict(dim=2, n=129, precision=0, rhs=("sine",), tol=0.0, cycles=10),
    "poisson3d_257_fp32ir": dict(dim=3, n=257, precision=1, rhs=("uniform", 0), tol=1e-8),
    "poisson2d_4097_fp32ir": dict(dim=2, n=4097, precision=1, rhs=("uniform", 0), tol=1e-8),
    # smooth log-normal coefficient in [1, 100] (seed 1), f ~ U[-1, 1] (seed 2)
    "varcoef3d_257_fp32ir": dict(dim=3, n=257, precision=1, rhs=("uniform", 2), k=1, tol=1e-8),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_k(w):
    import inputs

    return inputs.varcoef_k(w["n"], w["k"], dim=w["dim"]) if "k" in w else None


def make_rhs(w):
    import inputs

    if w["rhs"][0] == "sine":
        return inputs.sine_rhs(w["dim"], w["n"])
    return inputs.uniform_rhs(w["dim"], w["n"], w["rhs"][1])


def traffic_record(workload: str, tiles, key: str = "configs") -> dict | None:
    """HBM bytes per launch of a finest-level kernel (the sweep, key "configs",
    or the refinement pass, key "pass_configs", with the given tile geometry)
    from the committed rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, each
    calibrated on a 1 GiB copy), if they were taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get(key, {}).get(",".join(str(t) for t in tiles))


def cpu_baseline(w, gpu_steps: int, budget_s: float, min_steps: int = 3):
    """Time the oracle (as it stands) on one refinement step / one V-cycle of
    the same workload on this host; scale to the solve's step count.  Runs
    with the OpenMP thread count of the environment."""
    import numpy as np

    import oracle

    dim, n = w["dim"], w["n"]
    f = make_rhs(w)
    k = make_k(w)
    k32 = k.astype(np.float32) if k is not None else None
    u = np.zeros_like(f)
    threads = oracle.num_threads()
    t_steps = []
    t0 = time.perf_counter()

    def enough():
        el = time.perf_counter() - t0
        return el > budget_s or (len(t_steps) >= min_steps and el > 1.0)

    if w["precision"] == 1:
        e = np.zeros(f.shape, np.float32)
        while True:
            ts = time.perf_counter()
            u, r32, _ = oracle.ir_update(u, e, f, k=k)
            e = oracle.vcycle(np.zeros(f.shape, np.float32), r32, k=k32)
            t_steps.append(time.perf_counter() - ts)
            if enough():
                break
        sample = "FP64 refinement pass + FP32 V(2,2) cycle"
    elif w["precision"] == 2:
        e16, s_e, mx = None, 1.0, 0.0
        while True:
            ts = time.perf_counter()
            s_r = oracle.fp16_scale(mx)
            u, r16, _, mx = oracle.ir_update_f16(u, e16, s_e, f, s_r)
            e16, s_e = oracle.vcycle(np.zeros(f.shape, np.float16), r16), s_r
            t_steps.append(time.perf_counter() - ts)
            if enough():
                break
        sample = "FP64 refinement pass + binary16-storage V(2,2) cycle"
    else:
        while True:
            ts = time.perf_counter()
            u = oracle.vcycle(u, f, k=k)
            oracle.residual_norm(u, f, k=k)
            t_steps.append(time.perf_counter() - ts)
            if enough():
                break
        sample = "FP64 V(2,2) cycle + residual norm"
    t_step = float(np.median(t_steps))
    dof = (n - 2) ** dim
    t_solve = t_step * gpu_steps
    return {
        "value": dof / t_solve,
        "unit": "DoF/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{len(t_steps)} x ({sample}) on the {n}^{dim} workload, median {t_step:.3f} s per step, "
                  f"scaled by the {gpu_steps} steps of the solve",
    }


def cpu_info() -> dict:
    """CPU model and core counts of this host (lscpu), and the CPUs this process may use."""
    info = {"model": None, "sockets": None, "cores_per_socket": None, "threads_per_core": None}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
                "Thread(s) per core": "threads_per_core"}
        for line in out.splitlines():
            name, _, val = line.partition(":")
            if name.strip() in keys and info[keys[name.strip()]] is None:
                v = val.strip()
                info[keys[name.strip()]] = int(v) if v.isdigit() else v
    except (OSError, subprocess.SubprocessError):
        pass
    if isinstance(info["sockets"], int) and isinstance(info["cores_per_socket"], int):
        info["physical_cores"] = info["sockets"] * info["cores_per_socket"]
    else:
        info["physical_cores"] = None
    info["cpus_allowed"] = len(os.sched_getaffinity(0))
    return info


def cpu_baseline_legs(workload: str, gpu_steps: int, budget_s: float) -> dict:
    """The oracle on one thread and on all physical cores this process may use
    (OMP_PROC_BIND=close, OMP_PLACES=cores), each in a child process (which
    never touches the GPU).  A thread limit set in the environment
    (OMP_NUM_THREADS) caps the all-core leg."""
    info = cpu_info()
    allc = info["physical_cores"] or info["cpus_allowed"]
    allc = min(allc, info["cpus_allowed"])
    env_cap = os.environ.get("OMP_NUM_THREADS", "")
    if env_cap.isdigit() and int(env_cap) > 0:
        allc = min(allc, int(env_cap))
    legs = []
    for threads, budget, min_steps in ((1, budget_s * 0.6, 1), (allc, budget_s * 0.4, 3)):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_PROC_BIND="close", OMP_PLACES="cores")
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", "--workload", workload,
               "--gpu-steps", str(gpu_steps), "--cpu-budget", str(budget), "--cpu-min-steps", str(min_steps)]
        res = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
        if res.returncode != 0:
            raise RuntimeError(f"CPU leg with {threads} threads failed: {res.stderr[-2000:]}")
        leg = json.loads(res.stdout.strip().splitlines()[-1])
        leg["threads"] = threads
        legs.append(leg)
    main_leg = legs[-1]
    return {
        "value": main_leg["value"],
        "unit": "DoF/s",
        "cores": main_leg["cores"],
        "kind": "oracle",
        "sample": main_leg["sample"],
        "cpu_model": info["model"],
        "physical_cores": info["physical_cores"],
        "cpus_allowed": info["cpus_allowed"],
        "legs": [{"threads": g["threads"], "value": g["value"], "cores": g["cores"], "sample": g["sample"]}
                 for g in legs],
        "gpu_over_cpu_one_thread": None,
    }


def bench_batched(args, mg, torch):
    """512 independent 2D Poisson grids, edges drawn from {65, ..., 1025}, each
    solved to 1e-8 by FP32 V-cycles in FP64 refinement in one batched context;
    compared with solving the same grids one after another in FP64."""
    import numpy as np

    import inputs

    count = args.batch_count
    edges, rhs = inputs.batch_problem(count=count, seed=3)
    dof = sum((n - 2) ** 2 for n in edges)
    dev = torch.device("cuda:0")
    fs = [torch.from_numpy(f).to(dev) for f in rhs]
    us = [torch.zeros_like(f) for f in fs]
    del rhs
    log(f"[bench] batched: {count} grids, {dof} DoF, edges {sorted(set(edges))}")
    ctx = mg.mg_batch_setup([mg.Params(dim=2, n=n, precision=mg.PREC_FP32_IR) for n in edges])
    for _ in range(args.warmup):
        for u in us:
            u.zero_()
        mg.mg_batch_solve(ctx, us, fs, tol=1e-8, max_cycles=50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for u in us:
            u.zero_()
        st, cyc, stt = mg.mg_batch_solve(ctx, us, fs, tol=1e-8, max_cycles=50)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mg.mg_destroy(ctx)
    t_batch = (t1 - t0) / args.steps
    log(f"[bench] batched FP32-IR: {t_batch * 1e3:.2f} ms per batch, status {st}, cycles {min(cyc)}..{max(cyc)}")
    if args.no_fp64:
        return {"metric": "batched only", "value": dof / t_batch, "unit": "DoF/s", "ms_per_step": t_batch * 1e3}
    # the same grids one at a time, plain FP64 (one context per size)
    ctxs = {n: mg.Solver(mg.Params(dim=2, n=n, precision=mg.PREC_FP64)) for n in set(edges)}
    for u in us:
        u.zero_()
    for i, n in enumerate(edges[:8]):
        ctxs[n].solve(us[i], fs[i], tol=1e-8, max_cycles=50)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for i, n in enumerate(edges):
        us[i].zero_()
        ctxs[n].solve(us[i], fs[i], tol=1e-8, max_cycles=50)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for c in ctxs.values():
        c.close()
    t64 = tb - ta
    log(f"[bench] sequential FP64: {t64 * 1e3:.2f} ms for {count} solves")
    return {
        "metric": "fine-grid DoF/s + HBM GB/s %peak; solves/s & p99 latency at 1e-8 residual",
        "value": dof / t_batch,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"batched_2d_{count}", "grids": count, "dof": dof,
                   "edges": "uniform from {65,129,257,513,1025}, seed 3", "tol": 1e-8,
                   "solver": "batched FP32 V(2,2) RBGS in FP64 refinement, one launch per grid level"},
        "extra": {"solves_per_s": count / t_batch, "fp64_sequential_solves_per_s": count / t64,
                  "batched_over_fp64_sequential": t64 / t_batch,
                  "cycles_min_max": [min(cyc), max(cyc)]},
    }


def bench_serving(args, mg, torch):
    """Poisson arrival stream of mixed 2D/3D requests against the serving loop."""
    import numpy as np

    import inputs

    sp = mg.ServerParams(hbm_budget_bytes=args.serve_budget_gib << 30, max_slots=args.serve_slots,
                         max_n2d=2049, max_n3d=257, tol=1e-8, max_cycles=50)
    ctx = mg.mg_server_create(sp)
    # a pool of right-hand sides per size (requests of one size share a few seeds)
    pool = {}
    outs = {}  # one result buffer per size: every solution is copied back to the host

    def out_for(dim, n):
        if (dim, n) not in outs:
            outs[(dim, n)] = np.empty((n,) * dim)
        return outs[(dim, n)]

    def rhs_for(req):
        key = (req.dim, req.n, req.seed % 3)
        if key not in pool:
            pool[key] = inputs.uniform_rhs(req.dim, req.n, 5000 + req.seed % 3)
        return pool[key]

    dpool = {}  # device copies of the pooled right-hand sides (device-fed requests)

    def run(reqs, closed_loop=False, host=None, device=False):
        lat = []
        douts = {}  # device-fed request -> its solution array
        i = 0
        start = time.perf_counter()
        arrival_of = {}
        shape_of = {}
        clock = time.perf_counter
        while i < len(reqs) or arrival_of:
            now = clock() - start
            # closed loop: a fixed number of requests in flight, a new one per completion
            while i < len(reqs) and (len(arrival_of) < inflight if closed_loop else reqs[i].t_arrival <= now):
                t0 = clock()
                if device:
                    f = rhs_for(reqs[i])
                    key = (reqs[i].dim, reqs[i].n, reqs[i].seed % 3)
                    if key not in dpool:
                        dpool[key] = torch.from_numpy(f).to("cuda")
                        torch.cuda.synchronize()
                    ud = torch.empty_like(dpool[key])
                    rid = mg.mg_server_submit_device(ctx, dpool[key], ud)
                    douts[rid] = ud
                else:
                    rid = mg.mg_server_submit(ctx, rhs_for(reqs[i]))
                if host is not None:
                    host["submit"] += clock() - t0
                arrival_of[rid] = clock() if closed_loop else start + reqs[i].t_arrival
                shape_of[rid] = (reqs[i].dim, reqs[i].n)
                i += 1
            used, active, queued = mg.mg_server_info(ctx)
            if active == 0 and queued == 0 and not arrival_of and i < len(reqs):
                # idle: nothing admitted, queued or on its way back to the host
                time.sleep(max(0.0, reqs[i].t_arrival - (clock() - start)))
                continue
            t0 = clock()
            mg.mg_server_step(ctx)
            t1 = clock()
            for rid in mg.mg_server_poll(ctx):
                if device:
                    shape_of.pop(rid)
                    douts.pop(rid)
                    st, _, cyc, rr, _ = mg.mg_server_fetch(ctx, rid)
                else:
                    st, _, cyc, rr, _ = mg.mg_server_fetch(ctx, rid, out=out_for(*shape_of.pop(rid)))
                if st != 0:
                    raise RuntimeError(f"serving request {rid} ended with status {st}")
                tdone = clock()
                lat.append(tdone - arrival_of.pop(rid))
            if host is not None:
                host["step"] += t1 - t0
                host["poll_fetch"] += clock() - t1
                host["steps"] += 1
        span = clock() - start
        return np.array(lat), span

    # saturated throughput: closed loop with a fixed number of requests in flight
    inflight = args.serve_inflight
    sat_reqs = inputs.serving_requests(args.serve_requests, rate=1.0, seed=4)
    _ = run(sat_reqs[: max(8, args.serve_requests // 8)], closed_loop=True)  # warm pools and tuner
    host = {"submit": 0.0, "step": 0.0, "poll_fetch": 0.0, "steps": 0}
    lat, span = run(sat_reqs, closed_loop=True, host=host)
    mu_sat = len(sat_reqs) / span
    sat_p = [float(np.percentile(lat, q) * 1e3) for q in (50, 99)]
    log(f"[bench] serving: saturated {mu_sat:.1f} solves/s ({len(sat_reqs)} requests in {span:.2f} s, "
        f"{inflight} in flight, p50/p99 {sat_p[0]:.2f}/{sat_p[1]:.2f} ms); "
        f"host time in submit {host['submit']:.2f} s, step {host['step']:.2f} s ({host['steps']} calls), "
        f"poll+fetch {host['poll_fetch']:.2f} s")
    # the same closed loop fed from device memory (right-hand sides resident in
    # HBM, solutions copied device to device): no host staging of payloads
    host_d = {"submit": 0.0, "step": 0.0, "poll_fetch": 0.0, "steps": 0}
    lat_d, span_d = run(sat_reqs, closed_loop=True, host=host_d, device=True)
    mu_dev = len(sat_reqs) / span_d
    dev_p = [float(np.percentile(lat_d, q) * 1e3) for q in (50, 99)]
    log(f"[bench] serving, device-fed: saturated {mu_dev:.1f} solves/s, p50/p99 {dev_p[0]:.2f}/{dev_p[1]:.2f} ms; "
        f"host time in submit {host_d['submit']:.2f} s, step {host_d['step']:.2f} s, "
        f"poll+fetch {host_d['poll_fetch']:.2f} s")
    sweep = []
    for frac in (0.2, 0.4, 0.6, 0.8, 0.95):
        reqs = inputs.serving_requests(args.serve_requests, rate=frac * mu_sat, seed=4)
        lat, span = run(reqs)
        rec = {"lambda_frac": frac, "lambda": frac * mu_sat, "solves_per_s": len(reqs) / span,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}
        sweep.append(rec)
        log(f"[bench] serving lambda={rec['lambda']:.1f}/s: {rec['solves_per_s']:.1f} solves/s, "
            f"p50 {rec['p50_ms']:.2f} ms, p99 {rec['p99_ms']:.2f} ms")
    mg.mg_destroy(ctx)
    # the plain FP64 GPU solve of the same requests, one after another, with the
    # same host transfers (rhs up, solution back); one context per size
    seq = sat_reqs[: min(len(sat_reqs), args.serve_fp64_requests)]
    ctxs = {}
    for r in seq:
        if (r.dim, r.n) not in ctxs:
            ctxs[(r.dim, r.n)] = mg.Solver(mg.Params(dim=r.dim, n=r.n, precision=mg.PREC_FP64))

    def solve64(r):
        fd = torch.from_numpy(rhs_for(r)).to("cuda")
        u = torch.zeros_like(fd)
        ctxs[(r.dim, r.n)].solve(u, fd, tol=1e-8, max_cycles=50)
        out_for(r.dim, r.n)[...] = u.cpu().numpy()

    for r in seq[:8]:
        solve64(r)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for r in seq:
        solve64(r)
    torch.cuda.synchronize()
    fp64_rate = len(seq) / (time.perf_counter() - ta)
    for c in ctxs.values():
        c.close()
    log(f"[bench] plain FP64 GPU solves of the same requests one by one: {fp64_rate:.1f} solves/s "
        f"(served mix {mu_sat / fp64_rate:.1f}x)")
    mean_dof = float(np.mean([(r.n - 2) ** r.dim for r in sat_reqs]))
    return {
        "metric": "fine-grid DoF/s + HBM GB/s %peak; solves/s & p99 latency at 1e-8 residual",
        "value": mu_sat,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(sat_reqs),
        "warmup": 1,
        "ms_per_step": 1e3 / mu_sat,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serving_mix", "requests_per_lambda": args.serve_requests,
                   "saturated_inflight": args.serve_inflight,
                   "mix": "60% 2D edges {257,513,1025,2049}, 40% 3D edges {33,65,129,257}",
                   "arrivals": "exponential inter-arrival, seed 4", "tol": 1e-8,
                   "budget_gib": args.serve_budget_gib, "slots_per_dim": args.serve_slots},
        "extra": {"saturated_solves_per_s": mu_sat, "mean_dof_per_request": mean_dof,
                  "fp64_sequential_solves_per_s": fp64_rate, "fp64_sequential_requests": len(seq),
                  "served_over_fp64_sequential": mu_sat / fp64_rate,
                  "saturated_host_seconds": host, "saturated_p50_ms": sat_p[0], "saturated_p99_ms": sat_p[1],
                  "saturated_dof_per_s": mu_sat * mean_dof, "lambda_sweep": sweep,
                  "device_fed": {"saturated_solves_per_s": mu_dev, "saturated_dof_per_s": mu_dev * mean_dof,
                                 "saturated_p50_ms": dev_p[0], "saturated_p99_ms": dev_p[1],
                                 "saturated_host_seconds": host_d}},
    }


# Table 2's complex-diffusion rows: one V(2,2) cycle on N = 4096^2 (2D) and
# 256^3 (3D) cells; the paper's generated GPU code in double precision, in ms
# (GTX 680: the 1-core time divided by the GPU speed-up of the Double column).
CDIFF_PAPER_MS = {(2, 1): 9235 / 23.99, (2, 0): 7504 / 11.62, (3, 1): 8799 / 15.94, (3, 0): 9048 / 10.28}


def bench_cdiff(mg, torch, inputs, cycles: int = 5) -> dict:
    """Complex diffusion (implicit Euler, FAS with lagged diffusivity) at
    Table 2's sizes: the time of one FAS V(2,2) cycle (RBGS and Jacobi, FP64
    complex), inputs resident, and one whole time step to a 1e5 reduction."""
    import math

    out = {}
    for dim, n in ((2, 4096), (3, 256)):
        u0 = torch.from_numpy(inputs.noisy_image(dim, n, 11)).to("cuda")
        tau = 10.0 / n**2
        f = u0 * (1.0 / tau)
        cells = n**dim
        for sm, name in ((0, "rbgs"), (1, "jacobi")):
            ctx = mg.mg_cdiff_setup(dim, n, tau, math.pi / 30, 0.1, smoother=sm)
            u = u0.clone()
            mg.mg_cdiff_fas(ctx, u, f)  # warm
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(cycles):
                mg.mg_cdiff_fas(ctx, u, f)
            e1.record()
            torch.cuda.synchronize()
            ms_cycle = e0.elapsed_time(e1) / cycles
            u.copy_(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, cyc, hist = mg.mg_cdiff_run(ctx, u, 1, 1e-5, 10)
            t1 = time.perf_counter()
            mg.mg_destroy(ctx)
            paper = CDIFF_PAPER_MS[(dim, sm)]
            out[f"cdiff{dim}d_{n}_{name}"] = {
                "cells": cells, "ms_per_fas_cycle": ms_cycle, "cells_per_s": cells / (ms_cycle * 1e-3),
                "time_step": {"ms": (t1 - t0) * 1e3, "cycles": cyc[0], "status": st,
                              "reduction": hist[0][-1] / hist[0][0]},
                "paper_gtx680_fp64_ms_per_cycle": paper, "speedup_vs_paper_context": paper / ms_cycle}
            log(f"[bench] complex diffusion {dim}D {n}^{dim} {name}: {ms_cycle:.3f} ms per FAS V(2,2) cycle, "
                f"time step {cyc[0]} cycles in {(t1 - t0) * 1e3:.2f} ms")
        del u0, f, u
        torch.cuda.empty_cache()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson3d_513_fp32ir",
                    choices=sorted(WORKLOADS) + ["batched_2d", "serving_mix", "complex_diffusion"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 context solve")
    ap.add_argument("--no-fp16", action="store_true", help="skip the binary16-cycle solve of the same problem")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for the baseline")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-inflight", type=int, default=64, help="requests in flight in the saturated run")
    ap.add_argument("--serve-fp64-requests", type=int, default=300,
                    help="requests of the mix solved one by one in plain FP64 for comparison")
    ap.add_argument("--serve-budget-gib", type=int, default=48)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run the plain copy kernel over 1 GiB three times (counter calibration)")
    ap.add_argument("--no-cdiff", action="store_true",
                    help="skip the complex-diffusion leg of the default workload's line")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and serving legs of the default workload's line")
    ap.add_argument("--forms-requests", type=int, default=1000,
                    help="requests per arrival rate of the serving leg in the default workload's line")
    # child-process mode of the CPU baseline (never touches the GPU)
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--gpu-steps", type=int, default=7, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-min-steps", type=int, default=3, help=argparse.SUPPRESS)
    args = ap.parse_args(argv)
    if args.cpu_leg:
        print(json.dumps(cpu_baseline(WORKLOADS[args.workload], args.gpu_steps, args.cpu_budget,
                                      args.cpu_min_steps)), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1406_5369_amd as mg

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 2
    if args.workload == "batched_2d":
        print(json.dumps(bench_batched(args, mg, torch)), flush=True)
        mg.shutdown()
        return 0
    if args.workload == "serving_mix":
        print(json.dumps(bench_serving(args, mg, torch)), flush=True)
        mg.shutdown()
        return 0
    if args.workload == "complex_diffusion":
        import inputs

        print(json.dumps({"workload": "complex_diffusion", "unit": "ms per FAS V(2,2) cycle",
                          "legs": bench_cdiff(mg, torch, inputs, cycles=args.steps)}), flush=True)
        mg.shutdown()
        return 0
    w = WORKLOADS[args.workload]
    dim, n = w["dim"], w["n"]
    dof = (n - 2) ** dim
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] workload {args.workload}: dim={dim} n={n} dof={dof}")
    f = torch.from_numpy(make_rhs(w)).to(dev)
    max_cycles = w.get("cycles", 50)
    tol = w["tol"]

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            mg.mg_copy_kernel(dst, src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy kernel: 3 x 1 GiB")

    # measured HBM copy ceiling of this device: library copy kernel over 1 GiB (read + write)
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        mg.mg_copy_kernel(dst, src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(10):
        ev0.record()
        mg.mg_copy_kernel(dst, src)
        ev1.record()
        ev1.synchronize()
        best = min(best, ev0.elapsed_time(ev1))
    copy_gbps = 2.0 * (1 << 30) / (best * 1e-3) / 1e9
    del src, dst
    log(f"[bench] copy kernel ceiling: {copy_gbps:.0f} GB/s")

    # solution buffers, zeroed before the timed region (u0 = 0 for every step)
    nbuf = args.steps + args.warmup
    us = [torch.zeros_like(f) for _ in range(min(nbuf, 4))]
    k_host = make_k(w)
    kd = torch.from_numpy(k_host).to(dev) if k_host is not None else None
    op = mg.OP_VARCOEF_NODAL if kd is not None else mg.OP_LAPLACE
    params = mg.Params(dim=dim, n=n, precision=w["precision"], op=op, k=kd)
    solver = mg.Solver(params)
    stream = torch.cuda.current_stream()

    def one(i):
        u = us[i % len(us)]
        u.zero_()
        return solver.solve(u, f, tol=tol, max_cycles=max_cycles)

    for i in range(args.warmup):
        st, cyc, hist = one(i)
        log(f"[bench] warmup {i}: status={st} cycles={cyc} reduction={hist[-1] / hist[0]:.3e}")
    # timed region: K complete solves; the zeroing of u is part of each solve's setup
    mg.mg_prof_enable(solver.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = []
    for i in range(args.steps):
        st, cyc, hist = one(i)
        cycles.append(cyc)
        if st != mg.MG_OK:
            log(f"[bench] step {i}: status {st}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, sweep_ms = mg.mg_prof_read(solver.ctx, 0)
    pass_launches, pass_ms = mg.mg_prof_read(solver.ctx, 1)
    mg.mg_prof_enable(solver.ctx, False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = dof * args.steps / (t1 - t0)
    log(f"[bench] {args.steps} solves: {ms_per_step:.3f} ms/solve, cycles {cycles}, {value / 1e9:.3f} GDoF/s")
    # The timed solves above launch eagerly (the event brackets need it); the
    # same solves with the steps captured in HIP graphs, for comparison.
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for i in range(args.steps):
        one(i)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - tg0) * 1e3 / args.steps
    log(f"[bench] same solves with graph-captured steps: {ms_graph:.3f} ms/solve")

    # The two largest finest-level kernels, timed by the library with HIP events
    # on the solver's stream over the timed solves (launches of steps after a
    # solve finished, which do no work, not counted): the plain smoothing sweep
    # (reads u and f, writes u: 3 words per inner node, 4 with k) and the FP64
    # refinement pass (reads u, f, e, writes u, r: 32 B per inner node, +8 with
    # k) or, in FP64 solves, the norm pass (reads u, f: 16 B, +8 with k).  The
    # one with the larger total time is reported as the dominant kernel.
    word = {0: 8, 1: 4, 2: 2}[w["precision"]]
    var = kd is not None
    ir = w["precision"] in (1, 2)
    # refinement pass: FP64 u and f read, e read (float or binary16), FP64 u and r (float / binary16) written
    pass_bytes = (8 + 8 + 8 + 2 * word) if ir else 16

    def roof(kernel, blocks, note, n_launch, total_ms, bytes_per_launch, tr):
        avg_ms = total_ms / max(n_launch, 1)
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if n_launch else 0.0
        r = {"bound": "hbm", "kernel": kernel, "blocks": blocks, "note": note, "launches": n_launch,
             "avg_launch_ms": avg_ms, "total_ms": total_ms, "algorithmic_bytes_per_launch": bytes_per_launch,
             "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
             "copy_ceiling": copy_gbps, "frac_of_copy_ceiling": achieved / copy_gbps, "traffic": None}
        if tr and tr.get("kernel") == kernel and tr.get("blocks") == blocks:
            r["traffic"] = tr["bytes_per_launch"]
            r["traffic_ratio_to_algorithmic"] = tr["ratio_to_algorithmic"]
        return r

    by, zchunk, pd, wv = mg.mg_tile_config(solver.ctx, 0, 0)
    kname = sweep_kernel(dim, word, by, pd, var, wv)
    sweep_roof = roof(kname, sweep_blocks(dim, n, by, zchunk),
                      "finest-level RBGS sweeps that read the previous iterate (zero-iterate and fused-correction "
                      "variants excluded)", launches, sweep_ms, (4 if var else 3) * word * dof,
                      traffic_record(args.workload, (by, zchunk, pd, wv)))
    pby, pzc, ppd, pwv, _, ppr = mg.mg_tile_config(solver.ctx, 0, 2, with_order=True)
    nby, nzc, npd, nwv = mg.mg_tile_config(solver.ctx, 0, 6)
    if not ir and nzc > 0:
        # FP64 solves sum each cycle's residual norm in the next cycle's first
        # pre-smoothing sweep (reads u and f, writes the other buffer): the
        # event brackets time that sweep
        pass_roof = roof(sweep_kernel(dim, word, nby, npd, var, nwv, flags=4), sweep_blocks(dim, n, nby, nzc),
                         "finest-level FP64 first pre-smoothing sweep that also sums the residual norm of its "
                         "incoming iterate", pass_launches, pass_ms, (4 if var else 3) * word * dof,
                         traffic_record(args.workload, (nby, nzc, npd, nwv, "n")))
    else:
        pass_roof = roof(pass_kernel(dim, pby, ppd, var, ir, pwv, ppr, word=word),
                         pass_blocks(dim, n, pby, pzc, ppr),
                         ("finest-level FP64 refinement pass (u += e, r = f - A u, r to "
                          + ("FP32" if word == 4 else "scaled binary16") + ", norm partials)") if ir
                         else "finest-level FP64 residual-norm pass", pass_launches, pass_ms,
                         (pass_bytes + (8 if var else 0)) * dof,
                         traffic_record(args.workload, (pby, pzc, ppd, pwv) + (("p",) if ppr else ()),
                                        key="pass_configs"))
    if pass_roof["total_ms"] > sweep_roof["total_ms"]:
        roofline, other = pass_roof, sweep_roof
    else:
        roofline, other = sweep_roof, pass_roof
    if not other["launches"]:
        # no launch of that kernel in the timed solves (2D levels run their
        # sweeps as the fused pairs): nothing to report
        other = None
    log(f"[bench] finest sweep {sweep_roof['avg_launch_ms'] * 1e3:.1f} us x {launches}: "
        f"{sweep_roof['achieved']:.0f} GB/s; refinement/norm pass {pass_roof['avg_launch_ms'] * 1e3:.1f} us x "
        f"{pass_launches}: {pass_roof['achieved']:.0f} GB/s")

    extra = {"solves_per_s": args.steps / (t1 - t0), "cycles_per_solve": cycles[-1],
             "ms_per_solve_graph_captured": ms_graph,
             "kernel_source_hash": kernel_source_hash(),
             "roofline_other_kernel": other,
             "fine_tiles": {fam: mg.mg_tile_config(solver.ctx, 0, i, with_order=True) for i, fam in
                            enumerate(["smooth", "restrict", "norm_or_refinement", "smooth_zero_guess",
                                       "smooth_fused_correction", "smooth_fused_restriction",
                                       "smooth_with_norm", "two_smooths_from_zero", "two_post_smooths"])}}
    if not args.no_fp64 and w["precision"] == 1:
        s64 = mg.Solver(mg.Params(dim=dim, n=n, precision=mg.PREC_FP64, op=op, k=kd))
        u = us[0]
        u.zero_()
        s64.solve(u, f, tol=tol, max_cycles=max_cycles)  # warm
        reps = 3
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            u.zero_()
            st64, cyc64, h64 = s64.solve(u, f, tol=tol, max_cycles=max_cycles)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        s64.close()
        extra["fp64_solve"] = {"dof_per_s": dof * reps / (tb - ta), "ms_per_solve": (tb - ta) * 1e3 / reps,
                               "cycles": cyc64, "status": st64}
        extra["mixed_over_fp64_speedup"] = value / extra["fp64_solve"]["dof_per_s"]
        log(f"[bench] FP64 solve: {(tb - ta) * 1e3 / reps:.3f} ms, {cyc64} cycles")
    if not args.no_fp16 and w["precision"] == 1 and kd is None:
        # the binary16 form of the same solve: cycle fields stored as IEEE
        # binary16, float arithmetic, FP64 refinement; its finest sweep and
        # refinement pass timed by the library's event brackets
        u32 = us[0]
        u32.zero_()
        solver.solve(u32, f, tol=tol, max_cycles=max_cycles)
        s16 = mg.Solver(mg.Params(dim=dim, n=n, precision=mg.PREC_FP16_IR))
        u = us[1 % len(us)]
        u.zero_()
        s16.solve(u, f, tol=tol, max_cycles=max_cycles)  # warm
        reps = 3
        mg.mg_prof_enable(s16.ctx, True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            u.zero_()
            st16, cyc16, h16 = s16.solve(u, f, tol=tol, max_cycles=max_cycles)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        n16s, ms16s = mg.mg_prof_read(s16.ctx, 0)
        n16p, ms16p = mg.mg_prof_read(s16.ctx, 1)
        mg.mg_prof_enable(s16.ctx, False)
        s16_tiles = {fam: mg.mg_tile_config(s16.ctx, 0, i, with_order=True) for i, fam in
                     enumerate(["smooth", "restrict", "norm_or_refinement", "smooth_zero_guess",
                                "smooth_fused_correction"])}
        s16.close()
        rel = float(torch.linalg.vector_norm(u - u32) / torch.linalg.vector_norm(u32))
        sw_us = ms16s / max(n16s, 1) * 1e3
        ps_us = ms16p / max(n16p, 1) * 1e3
        extra["fp16_solve"] = {
            "dof_per_s": dof * reps / (tb - ta), "ms_per_solve": (tb - ta) * 1e3 / reps, "cycles": cyc16,
            "status": st16, "final_rel_residual": h16[-1] / h16[0],
            "rel_diff_vs_fp32ir_solution": rel,
            "finest_sweep": {"avg_launch_us": sw_us, "launches": n16s,
                             "achieved_gbps": 3 * 2 * dof / (sw_us * 1e-6) / 1e9 if n16s else None},
            "finest_refinement_pass": {"avg_launch_us": ps_us, "launches": n16p,
                                       "achieved_gbps": 28 * dof / (ps_us * 1e-6) / 1e9 if n16p else None},
            "fine_tiles": s16_tiles}
        extra["fp16_over_fp32ir_speedup"] = extra["fp16_solve"]["dof_per_s"] / value
        log(f"[bench] binary16 solve: {(tb - ta) * 1e3 / reps:.3f} ms, {cyc16} steps, "
            f"|u16 - u32| / |u32| = {rel:.2e}")
    solver.close()
    del us, f, kd
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # The other forms of the solver in the same line (default workload only):
    # the 512-grid batch and the serving sweep, each a shorter run of its own
    # workload (--workload batched_2d / serving_mix run them in full).
    if args.workload == "poisson3d_513_fp32ir" and not args.no_forms:
        bargs = argparse.Namespace(**vars(args))
        bargs.steps, bargs.warmup, bargs.no_fp64 = 3, 1, False
        b = bench_batched(bargs, mg, torch)
        extra["batched_2d"] = {"workload": b["config"]["workload"], "grids": b["config"]["grids"],
                               "dof": b["config"]["dof"], "ms_per_batch": b["ms_per_step"],
                               "dof_per_s": b["value"], "batches_timed": bargs.steps, **b["extra"]}
        torch.cuda.empty_cache()
        sargs = argparse.Namespace(**vars(args))
        sargs.serve_requests = args.forms_requests
        sargs.serve_fp64_requests = min(args.serve_fp64_requests, 200)
        sv = bench_serving(sargs, mg, torch)
        extra["serving_mix"] = {"requests_per_lambda": sargs.serve_requests, "config": sv["config"],
                                "saturated_solves_per_s": sv["value"], **sv["extra"]}
        torch.cuda.empty_cache()
    if args.workload == "poisson3d_513_fp32ir" and not args.no_cdiff:
        import inputs

        extra["complex_diffusion"] = bench_cdiff(mg, torch, inputs)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline (1 thread, all physical cores) ...")
        cpu = cpu_baseline_legs(args.workload, cycles[-1], args.cpu_budget)
        cpu["gpu_over_cpu_one_thread"] = value / cpu["legs"][0]["value"]
        log(f"[bench] CPU oracle ({cpu['cpu_model']}): " + ", ".join(
            f"{g['value'] / 1e6:.3f} MDoF/s on {g['cores']} threads" for g in cpu["legs"]))

    out = {
        "metric": "fine-grid DoF/s + HBM GB/s %peak; solves/s & p99 latency at 1e-8 residual",
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f64", 1: "f32+f64", 2: "f16+f32+f64"}[w["precision"]],
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "dim": dim,
            "n": n,
            "dof": dof,
            "tol": tol,
            "solver": "V(2,2) RBGS, full weighting, linear interpolation, exact 3-point coarsest solve"
                      + {0: ", FP64", 1: ", FP32 cycles in FP64 iterative refinement",
                         2: ", binary16-storage cycles (FP32 arithmetic) in FP64 iterative refinement"}[
                          w["precision"]],
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    mg.shutdown()
    return 0


if __name__ == "__main__":
    sys.exit(main())
