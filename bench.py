"""Throughput benchmark of the FLD radiation-energy step on one MI355X.

Default workload: the 2D 1024 x 1024 FP64 configuration with gas -- every step
is one implicit diffusion solve to a 1e-10 relative residual followed by the
implicit gas-radiation energy exchange, on seeded synthetic fields that stay
resident in HBM.  ``--steps K`` steps are timed after ``--warmup W`` untimed
ones (the trajectory continues through both).

One JSON line is printed: cell-updates/s (cells x steps / wall time), per-step
latency percentiles, the roofline of the dominant kernel (timed with HIP events
right after the timed region, on the same stream) and the FP64 CPU oracle timed
on one step of the same grid on this host's cores.

``--config c5`` runs the served stream instead: Poisson arrivals of mixed 2D and
3D solves submitted to the continuous-batching server on their schedule, with
throughput, offered load and p50/p99 request latency.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--requests", type=int, default=384, help="c5: requests in the stream")
    ap.add_argument("--rate", type=float, default=2000.0, help="c5: mean arrival rate (1/s)")
    ap.add_argument("--arena-gb", type=float, default=32.0, help="c5: server arena")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=200)
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1, 2],
                    help="launch shape: 0 defaults, 1 autotuner (cached), 2 re-time")
    ap.add_argument("--fmg", type=int, default=1, choices=[0, 1],
                    help="1: each step starts with a full-multigrid cycle")
    ap.add_argument("--fmg-depths", type=int, default=None,
                    help="full-multigrid start: V-cycles on the finest k levels only (0 = all; "
                         "default: the library's)")
    ap.add_argument("--coarse-op", default="rediscretised", choices=["rediscretised", "galerkin"],
                    help="coarse-level operator of the multigrid hierarchy")
    ap.add_argument("--nu", type=int, nargs=2, default=(2, 2), metavar=("NU1", "NU2"),
                    help="red-black sweeps before and after the coarse correction")
    ap.add_argument("--nu-coarse", type=int, default=0,
                    help="red-black sweeps before and after the correction on the coarse levels "
                         "(0 = nu1 and nu2, as on the finest level)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dominant_kernel(fld, ndim: int, word: int, fused: bool, fused3: bool):
    """The kernel that dominates a step and its algorithmic bytes per cell of level 0.

    2D (fused level kernels): the level-0 up pass reads the down pass's iterate,
    b, both face arrays and a quarter-size coarse correction, and writes x:
    (5 + 1/4) words.  3D fused sweeps: one whole red-black sweep reads x, b and
    the three face arrays once and writes x: 6 words.  3D per-colour kernels:
    one half sweep reads x of every cell, b of the updated half, every face
    weight (each face touches one cell of each colour) and writes x of the
    updated half: (2 + d) words.
    """
    if ndim == 2 and fused:
        return fld.FLD_KERNEL_UP, "k_up2", word * 5 + word / 4
    if ndim == 3 and fused3:
        return fld.FLD_KERNEL_SWEEP3, "k_sweep3", word * 6
    return fld.FLD_KERNEL_SMOOTH, "k_smooth", word * (2 + ndim)


def time_moments(fld, plan, grids, E, K, stream, reps: int = 20):
    """Time fld_radiation_moments with every output and a synthetic velocity field (HIP
    events on the bench stream, after the timed steps).  Algorithmic bytes per cell:
    E, kappa rho and the d velocity components read; d flux, d force, f, d(d+1)/2
    pressure components, the tiring work and E_out written (8 B each)."""
    import torch
    import workloads as W
    nd = grids[0].E.ndim
    v = [[torch.from_numpy(W.smooth_field(g.E.shape, 4242 + 10 * i + a)).to(E[0].device) for a in range(g.E.ndim)]
         for i, g in enumerate(grids)]
    outs = []
    for e in E:
        d = e.dim()
        outs.append({"F": [torch.empty_like(e) for _ in range(d)], "f_r": [torch.empty_like(e) for _ in range(d)],
                     "edd": torch.empty_like(e), "P": [torch.empty_like(e) for _ in range(d * (d + 1) // 2)],
                     "tiring": torch.empty_like(e), "E_out": torch.empty_like(e)})
    dts = [g.dt for g in grids]
    call = lambda: fld.fld_radiation_moments(plan.handle, E, K, outs, v=v, dt=dts, stream=stream)
    call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    cells = sum(g.E.size for g in grids)
    bpc = 8 * ((2 + nd) + (nd + nd + 1 + nd * (nd + 1) // 2 + 2))
    gbs = bpc * cells / (us * 1e-6) / 1e9
    return {"kernel": "k_moments", "us_per_call": us, "cells": cells, "bytes_per_cell": bpc,
            "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS}


def time_imex(fld, plan, grids, E, eps, rho, kap, gas, stream, reps: int = 5):
    """Time fld_imex_step (midpoint scheme, with a synthetic velocity: tiring and
    exchange in the explicit stages, one implicit half step) on copies of the
    post-benchmark state, wall clock around synchronous calls."""
    import torch
    import workloads as W
    v = [[torch.from_numpy(W.smooth_field(g.E.shape, 4343 + 10 * i + a)).to(E[0].device) for a in range(g.E.ndim)]
         for i, g in enumerate(grids)]
    dts = [g.dt for g in grids]
    out = {}
    for scheme in ("euler", "midpoint"):
        Ec = [e.clone() for e in E]
        ec = [x.clone() for x in eps]
        cyc = []

        def call():
            rc, st = plan.imex_step(Ec, ec, rho, kap, dts, gas=gas, scheme=scheme, v=v, stream=stream, check=False)
            if rc != 0:
                raise RuntimeError(f"fld_imex_step failed: {fld.fld_strerror(rc)}")
            cyc.append(max(s["cycles"] for s in st))
        call()
        torch.cuda.synchronize()
        cyc.clear()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / reps
        cells = sum(g.E.size for g in grids)
        out[scheme] = {"ms_per_step": dt_s * 1e3, "cell_updates_per_s": cells / dt_s,
                       "vcycles": float(np.mean(cyc)), "steps": reps}
    return out


def measured_traffic(cfg: str, kname: str, launch: dict):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    record kept under profiles/ (copy-calibrated), or None when there is no record for this
    workload and launch shape, or kernels.hip has changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2104_03968_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    keys = ("tile_rows", "tile_wide", "max_blocks", "tile_depth", "fused3_levels", "tile_rows_coarse", "tile_rows_up")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_record: "):
                continue
            rec = json.loads(line[len("traffic_record: "):])
            if (rec.get("config") == cfg and rec.get("kernel", "").startswith(kname + "<")
                    and rec.get("kernels_sha256") == sha
                    and all(rec.get("launch", {}).get(k) == launch.get(k) for k in keys)):
                return float(rec["bytes_per_launch"])
    return None


def cpu_baseline(g, steps_gas: bool):
    import oracle as O
    t0 = time.perf_counter()
    x, info = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h, g.c)
    if steps_gas:
        O.exchange(x, g.eps, g.rho, g.kappa, g.dt, g.c, g.a_r, g.c_v)
    t = time.perf_counter() - t0
    return t, info


def serve_stream(args):
    """The served Poisson stream through the request server."""
    import threading
    import torch
    import workloads as W
    import paper_2104_03968_amd as fld

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    reqs = W.c5_stream(args.requests, rate=args.rate)
    log(f"bench c5: generating {len(reqs)} requests on the device")
    inputs = []
    for r in reqs:
        g = r.inputs(backend="torch", device=dev)
        inputs.append((g.E.contiguous(), g.kappa_rho.contiguous(), g.h))
    torch.cuda.synchronize()
    precision = fld.FLD_PREC_FP64 if args.precision == "fp64" else fld.FLD_PREC_MIXED
    srv = fld.Server(int(args.arena_gb * (1 << 30)), precision=precision, rtol=1e-10)
    # warm-up: one small request of each dimension (compiles nothing, but pages in the code)
    for shape in ((128, 128), (32, 32, 32)):
        g = W.random_grid(shape, 1, 1e-3, backend="torch", device=dev)
        t = srv.submit(g.E.contiguous(), g.kappa_rho.contiguous(), g.dt, h=g.h)
        srv.wait(t, 60.0)
        srv.release(t)
    tickets = [None] * len(reqs)
    submit_wall = [0.0] * len(reqs)

    def client():
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            while time.perf_counter() - t0 < r.t_arrival:
                time.sleep(max(0.0, min(1e-3, r.t_arrival - (time.perf_counter() - t0))))
            E, K, h = inputs[i]
            tickets[i] = srv.submit(E, K, r.dt, h=h)
            submit_wall[i] = time.perf_counter()

    th = threading.Thread(target=client)
    t_start = time.perf_counter()
    th.start()
    lat, done_t, cycles, statuses = [], [], [], []
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(1e-4)
        rc, res = srv.wait(tickets[i], 600.0)
        statuses.append(rc)
        lat.append(res.t_done - res.t_submit)
        done_t.append(res.t_done)
        cycles.append(res.stats.cycles)
        srv.release(tickets[i])
    th.join()
    t_end = time.perf_counter()
    info = srv.info()
    srv.close()
    cells = sum(r.cells for r in reqs)
    makespan = t_end - t_start
    offered = cells / max(reqs[-1].t_arrival, 1e-9)
    out = {
        "metric": "cell-updates/s of implicit FLD step at 1e-10 residual; p50/p99 solve latency",
        "value": cells / makespan,
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": len(reqs), "warmup": 2,
        "ms_per_step": makespan / len(reqs) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == fld.FLD_PREC_FP64 else "f32-in-f64",
        "data": "synthetic",
        "config": {"workload": (f"served stream: {len(reqs)} Poisson arrivals at {args.rate:.0f}/s of 2D "
                                "128^2..1024^2 and 3D 32^3..192^3 FLD solves, dt U[1e-4,1e-2], rtol 1e-10, "
                                "continuous batching, arena admission"),
                   "cells": cells, "arena_gb": args.arena_gb},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "offered_cell_updates_per_s": offered,
        "makespan_s": makespan,
        "failed": int(sum(1 for s_ in statuses if s_ != 0)),
        "vcycles_per_request": float(np.mean(cycles)),
        "server": {"rounds": info["rounds"], "completed": info["completed"]},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.config == "c5" and args.gpus == 1:
        serve_stream(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        log("bench.py: only single-GPU runs are supported (the workload is one GPU's share)")
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2104_03968_amd as fld

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = args.config
    prec = args.precision or ("mixed" if cfg == "c3" else "fp64")
    precision = fld.FLD_PREC_MIXED if prec == "mixed" else fld.FLD_PREC_FP64
    log(f"bench: building inputs for {cfg} ({prec})")

    has_gas = False
    if cfg == "c1":
        grids = [W.pulse_2d()]
        workload = "2D 64x64 Gaussian pulse, kappa*rho=10, one backward-Euler FLD step"
    elif cfg == "c2":
        grids = [W.c2_inputs(1024)]
        has_gas = True
        workload = ("2D 1024x1024 FP64 FLD step + implicit gas-radiation exchange, log10(kappa*rho) "
                    "in [-2,2] (32 Fourier modes), log-normal E (sigma=1), dt=1e-3, rtol=1e-10")
    elif cfg == "c3":
        grids = [W.c3_inputs(256)]
        workload = ("3D 256^3 FLD step, the 2D 1024^2 field recipe in 3D, dt=1e-3, rtol=1e-10, "
                    + ("mixed (FP32 V-cycles in FP64 defect correction)" if prec == "mixed" else "fp64"))
    else:
        lay = W.c4_layout()
        grids = [W.c4_grid(j, n, dt) for j, (n, dt) in enumerate(lay)]
        workload = "512 independent 2D grids, sides U{64..512 step 32}, dt U[1e-4,1e-2], one launch per phase"
    ncells = sum(g.E.size for g in grids)
    shapes = [g.E.shape for g in grids]
    plan = fld.Plan(shapes, h=[g.h for g in grids], precision=precision, rtol=1e-10, c=grids[0].c,
                    autotune=args.autotune, fmg=args.fmg, coarse_op=args.coarse_op,
                    nu1=args.nu[0], nu2=args.nu[1], nu_coarse=args.nu_coarse, **({} if args.fmg_depths is None else {"fmg_depths": args.fmg_depths}))
    tuning = plan.tuning()
    log(f"bench: launch shape {tuning}")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    E = [to(g.E) for g in grids]
    K = [to(g.kappa_rho) for g in grids]
    dts = [g.dt for g in grids]
    if has_gas:
        eps = [to(g.eps) for g in grids]
        rho = [to(g.rho) for g in grids]
        kap = [to(g.kappa) for g in grids]
        gas = fld.fld_gas_default(c=grids[0].c, a_rad=grids[0].a_r, c_v=grids[0].c_v)
    stream = torch.cuda.current_stream()

    cycles = []

    def one_step():
        rc, st = plan.step(E, K, E, dts, stream=stream, check=False)
        if rc != 0:
            raise RuntimeError(f"fld_step failed: {fld.fld_strerror(rc)} {st[:2]}")
        if has_gas:
            plan.exchange(E, eps, rho, kap, dts, gas, stream=stream)
        cycles.append(max(s["cycles"] for s in st))
        return st

    log(f"bench: {len(grids)} grid(s), {ncells} cells; warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    cycles.clear()
    lat = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st = one_step()
        if has_gas:
            stream.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = ncells * args.steps / elapsed
    log(f"bench: {args.steps} steps in {elapsed:.4f} s -> {value:.4e} cell-updates/s, cycles {cycles}")
    if has_gas:
        rc, nbis = plan.exchange_status(stream)
        assert rc == 0, "exchange rejected cells"

    # dominant kernel at level 0, timed with HIP events on the same stream
    ndim = len(shapes[0])
    word = 4 if precision == fld.FLD_PREC_MIXED else 8
    kid, kname, bpc = dominant_kernel(fld, ndim, word, bool(plan.opts.fused), bool(tuning["fused3"]))
    ms, cells = plan.profile(kid, 0, args.profile_reps, stream)
    achieved = bpc * cells / (ms * 1e-3) / 1e9
    log(f"bench: level-0 {kname} {ms * 1e3:.2f} us for {cells} cells ({bpc} B/cell) -> {achieved:.0f} GB/s")

    out = {
        "metric": "cell-updates/s of implicit FLD step at 1e-10 residual; p50/p99 solve latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == fld.FLD_PREC_FP64 else "f32-in-f64",
        "data": "synthetic",
        "config": {"workload": workload, "cells": ncells, "grids": len(grids), "precision": prec,
                   "rtol": 1e-10, "fmg": plan.opts.fmg, "fmg_depths": plan.opts.fmg_depths, "coarse_op": args.coarse_op,
                   "nu": [plan.opts.nu1, plan.opts.nu2], "nu_coarse": plan.opts.nu_coarse,
                   "launch": {k: tuning[k] for k in ("tile_rows", "tile_wide", "max_blocks", "tile_depth",
                                                     "fused3_levels", "tile_rows_coarse", "tile_rows_up",
                                                     "source")}},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "vcycles_per_step": float(np.mean(cycles)) if cycles else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(cfg, kname, tuning),
                     "kernel": f"{kname} level 0 ({cells} cells, {bpc} B/cell, {ms * 1e3:.2f} us/launch)"},
    }
    out["radiation_moments"] = time_moments(fld, plan, grids, E, K, stream)
    if has_gas:
        log("bench: timing the IMEX step (tiring + exchange + implicit diffusion)")
        out["imex_step"] = time_imex(fld, plan, grids, E, eps, rho, kap, gas, stream)
    if not args.no_cpu_baseline:
        g0 = grids[0] if cfg != "c4" else grids[0]
        log("bench: timing the FP64 CPU oracle on one step of the first grid")
        t, info = cpu_baseline(g0, has_gas)
        out["cpu_baseline"] = {"value": g0.E.size / t, "unit": "cell-updates/s", "cores": 1,
                               "kind": "oracle",
                               "sample": (f"one FLD step of a {'x'.join(map(str, g0.E.shape))} grid "
                                          f"({info.method}, {info.iterations} iterations, {t:.1f} s; "
                                          "scipy sparse + numpy, single-threaded)"),
                               "host_cpus": os.cpu_count()}
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
