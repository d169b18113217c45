"""Throughput benchmark of the FLD radiation-energy step on one MI355X.

Default workload: the 3D 256^3 FP64 configuration -- every step is one
implicit backward-Euler diffusion solve to a 1e-10 relative residual on seeded
synthetic fields that stay resident in HBM.  ``--steps K`` steps are timed
after ``--warmup W`` untimed ones (the trajectory continues through both).

One JSON line is printed: cell-updates/s (cells x steps / wall time), per-step
latency percentiles, the roofline of the dominant kernel (timed with HIP events
right after the timed region, on the same stream), the effective bandwidth of a
whole outer iteration and of its multigrid V-cycle (algorithmic bytes of every
kernel over the pass's time), and the FP64 CPU oracle timed on a bounded sample
of the workload on this host's cores.  Extras (``--no-extras`` skips them): the
same grid in the other precision with its speed-up, five steps of both
precisions certified against the FP64 oracle, and the 2D 1024^2 step with gas.

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
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--requests", type=int, default=384, help="c5: requests in the stream")
    ap.add_argument("--rate", type=float, default=2000.0, help="c5: mean arrival rate (1/s)")
    ap.add_argument("--arena-gb", type=float, default=32.0, help="c5: server arena")
    ap.add_argument("--batch", type=int, default=64,
                    help="c5: requests per plan of the batched comparison on the same requests")
    ap.add_argument("--cycles-per-round", type=int, default=None,
                    help="c5: V-cycles between the server's admission / retirement points")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default fp64 (the served stream: mixed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline: no other precision, error certificates, 1024^2 line, "
                         "moments or IMEX timings")
    ap.add_argument("--krylov", type=int, default=1, choices=[0, 1],
                    help="1: V-cycle-preconditioned CG; 0: plain V-cycles (defect correction)")
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
    ap.add_argument("--nu-coarse", type=int, default=None,
                    help="red-black sweeps before and after the correction on the coarse levels "
                         "(0 = nu1 and nu2, as on the finest level; default: the library's)")
    ap.add_argument("--fused", type=int, default=None, choices=[0, 1, 2, 3],
                    help="2D fused level passes: 2 = LDS tiles only, 3 = row-marching windows wherever "
                         "fused, 0 = per-colour kernels (default: the library's rule)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dominant_kernel(fld, ndim: int, word: int, fused: bool, fused3: bool, march: bool = False):
    """The kernel that dominates a step and its algorithmic bytes per cell of level 0.

    2D (fused level kernels, LDS tiles or row-marching windows): the level-0 up pass
    reads the down pass's iterate, b, both face arrays and a quarter-size coarse
    correction, and writes x: (5 + 1/4) words.  3D fused sweeps: one whole red-black sweep reads x, b and
    the three face arrays once and writes x: 6 words.  3D per-colour kernels:
    one half sweep reads x of every cell, b of the updated half, every face
    weight (each face touches one cell of each colour) and writes x of the
    updated half: (2 + d) words.
    """
    if ndim == 2 and fused:
        return fld.FLD_KERNEL_UP, "k_march2" if march else "k_up2", word * 5 + word / 4
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


def measured_traffic(cfg: str, kname: str, ctype: str, launch: dict):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    record kept under profiles/ (copy-calibrated), or None when there is no record for this
    workload and launch shape, or kernels.hip has changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2104_03968_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    # the launch parameters the dominant kernel's own dispatch depends on
    keys = {"k_sweep3": ("tile_depth", "max_blocks"),
            "k_up2": ("tile_rows_up", "tile_wide", "max_blocks"),
            "k_march2": ("max_blocks",),
            "k_smooth": ("max_blocks",)}.get(kname, ("tile_rows", "tile_wide", "max_blocks", "tile_depth",
                                                    "fused3_levels", "tile_rows_coarse", "tile_rows_up"))
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_record: "):
                continue
            rec = json.loads(line[len("traffic_record: "):])
            if (rec.get("config") == cfg and rec.get("kernel", "").startswith(f"{kname}<{ctype}")
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
    sopts = {} if args.cycles_per_round is None else {"cycles_per_round": args.cycles_per_round}
    srv = fld.Server(int(args.arena_gb * (1 << 30)), precision=precision, rtol=1e-10, **sopts)
    # warm-up: one small request of each dimension (compiles nothing, but pages in the code)
    for shape in ((128, 128), (32, 32, 32)):
        g = W.random_grid(shape, 1, 1e-3, backend="torch", device=dev)
        torch.cuda.synchronize()
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
    lat, wait, done_t, cycles, statuses = [], [], [], [], []
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(1e-4)
        rc, res = srv.wait(tickets[i], 600.0)
        statuses.append(rc)
        lat.append(res.t_done - res.t_submit)
        wait.append(res.t_admit - res.t_submit)
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
    batched = None if args.no_extras else batched_same_requests(reqs, inputs, precision, args.batch)
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
        "admission_wait_ms": {"p50": float(np.percentile(wait, 50) * 1e3),
                              "p99": float(np.percentile(wait, 99) * 1e3)},
        "offered_cell_updates_per_s": offered,
        "achieved_over_offered": (cells / makespan) / offered,
        "batched_same_requests": batched,
        "makespan_s": makespan,
        "failed": int(sum(1 for s_ in statuses if s_ != 0)),
        "vcycles_per_request": float(np.mean(cycles)),
        "server": {"rounds": info["rounds"], "completed": info["completed"]},
    }
    print(json.dumps(out), flush=True)


def batched_same_requests(reqs, inputs, precision, batch):
    """The same requests as back-to-back batched steps: consecutive groups of `batch`
    (in arrival order) in one multi-grid plan each, with the server's solver options
    (rtol 1e-10, plain starts, CG).  Plans are built and warmed outside the clock; the
    figure is the cells over the summed step times, the rate the batched path reaches
    on this stream when nothing waits for arrivals."""
    import torch
    import paper_2104_03968_amd as fld
    total_s, steps = 0.0, 0
    for i0 in range(0, len(reqs), batch):
        grp = range(i0, min(i0 + batch, len(reqs)))
        plan = fld.Plan([tuple(inputs[i][0].shape) for i in grp], h=[inputs[i][2] for i in grp],
                        precision=precision, rtol=1e-10, fmg=0, autotune=0)
        E = [inputs[i][0] for i in grp]
        K = [inputs[i][1] for i in grp]
        out = [torch.empty_like(e) for e in E]
        dts = [reqs[i].dt for i in grp]
        plan.step(E, K, out, dts)                   # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(E, K, out, dts)
        torch.cuda.synchronize()
        total_s += time.perf_counter() - t0
        steps += 1
        plan.close()
        del out
    cells = sum(r.cells for r in reqs)
    log(f"bench c5: batched reference {steps} plans of <= {batch} requests, {total_s:.3f} s of steps")
    return {"value": cells / total_s, "unit": "cell-updates/s", "batch": batch, "plans": steps,
            "step_s": total_s}


def host_info(threads_used: int) -> dict:
    """CPU model, affinity and thread settings of this host (for the CPU baseline)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
           if os.environ.get(k) is not None}
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "sched_affinity": affinity,
            "thread_env": env, "threads_used": threads_used}


def certified_error(g_host, E_n, x):
    """Relative residual of the device's step under the oracle's own FP64 operator (built
    from E_n) and the bound q_b * residual it gives on the error against the oracle's
    exact step (A is SPD with lambda_min >= 1 and conserves the mean)."""
    import oracle as O
    D = O.diffusion_coefficient(E_n, g_host.kappa_rho, g_host.h, g_host.c)
    w = O.face_weights(D, g_host.dt, g_host.h)
    r = E_n - O.apply_operator(w, x)
    rel = float(np.linalg.norm(r) / np.linalg.norm(E_n))
    return rel, O.q_b(E_n) * rel


def build_config(W, cfg: str):
    """The seeded inputs of a configuration, whether it has gas, and its description."""
    if cfg == "c1":
        return [W.pulse_2d()], False, "2D 64x64 Gaussian pulse, kappa*rho=10, one backward-Euler FLD step"
    if cfg == "c2":
        return ([W.c2_inputs(1024)], True,
                "2D 1024x1024 FP64 FLD step + implicit gas-radiation exchange, log10(kappa*rho) "
                "in [-2,2] (32 Fourier modes), log-normal E (sigma=1), dt=1e-3, rtol=1e-10")
    if cfg == "c3":
        return ([W.c3_inputs(256)], False,
                "3D 256^3 FLD step, log10(kappa*rho) in [-2,2] and log-normal E (sigma=1) from "
                "32 Fourier modes, dt=1e-3, rtol=1e-10")
    lay = W.c4_layout()
    return ([W.c4_grid(j, n, dt) for j, (n, dt) in enumerate(lay)], False,
            "512 independent 2D grids, sides U{64..512 step 32}, dt U[1e-4,1e-2], one launch per phase")


def run_timed(fld, torch, args, cfg, grids, has_gas, precision, dev, steps, warmup, want_roofline=True):
    """Time `steps` steps (after `warmup`) of one configuration in one precision.
    Returns the measurement dict, the plan (open) and the device state."""
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], precision=precision, rtol=1e-10,
                    c=grids[0].c, autotune=args.autotune, fmg=args.fmg, coarse_op=args.coarse_op,
                    nu1=args.nu[0], nu2=args.nu[1], krylov=args.krylov,
                    **({} if args.fmg_depths is None else {"fmg_depths": args.fmg_depths}),
                    **({} if args.nu_coarse is None else {"nu_coarse": args.nu_coarse}),
                    **({} if args.fused is None else {"fused": args.fused}))
    tuning = plan.tuning()
    log(f"bench {cfg}: launch shape {tuning}")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    E = [to(g.E) for g in grids]
    K = [to(g.kappa_rho) for g in grids]
    dts = [g.dt for g in grids]
    st_ = {}
    if has_gas:
        st_["eps"] = [to(g.eps) for g in grids]
        st_["rho"] = [to(g.rho) for g in grids]
        st_["kap"] = [to(g.kappa) for g in grids]
        st_["gas"] = fld.fld_gas_default(c=grids[0].c, a_rad=grids[0].a_r, c_v=grids[0].c_v)
    stream = torch.cuda.current_stream()
    cycles = []

    def one_step():
        rc, st = plan.step(E, K, E, dts, stream=stream, check=False)
        if rc != 0:
            raise RuntimeError(f"fld_step failed: {fld.fld_strerror(rc)} {st[:2]}")
        if has_gas:
            plan.exchange(E, st_["eps"], st_["rho"], st_["kap"], dts, st_["gas"], stream=stream)
        cycles.append(max(s["cycles"] for s in st))
        return st

    ncells = sum(g.E.size for g in grids)
    log(f"bench {cfg}: {len(grids)} grid(s), {ncells} cells; warmup {warmup}")
    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    cycles.clear()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        one_step()
        if has_gas:
            stream.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = ncells * steps / elapsed
    log(f"bench {cfg}: {steps} steps in {elapsed:.4f} s -> {value:.4e} cell-updates/s, cycles {cycles}")
    if has_gas:
        rc, nbis = plan.exchange_status(stream)
        assert rc == 0, "exchange rejected cells"
    out = {"value": value, "ms_per_step": elapsed / steps * 1e3,
           "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
           "vcycles_per_step": float(np.mean(cycles)) if cycles else None, "tuning": tuning}
    if want_roofline:
        ndim = len(grids[0].E.shape)
        word = 4 if precision == fld.FLD_PREC_MIXED else 8
        o = plan.opts
        nuc = o.nu_coarse or 0
        # the fused 2D level kernels take 1 to 3 sweeps; other counts run per colour
        fused2 = bool(o.fused) and all(1 <= v <= 3 for v in (o.nu1, o.nu2, nuc or o.nu1, nuc or o.nu2))
        kid, kname, bpc = dominant_kernel(fld, ndim, word, fused2, bool(tuning["fused3"]),
                                          tuning.get("march_levels", 0) > 0)
        ms, cells = plan.profile(kid, 0, args.profile_reps, stream)
        achieved = bpc * cells / (ms * 1e-3) / 1e9
        log(f"bench {cfg}: level-0 {kname} {ms * 1e3:.2f} us for {cells} cells ({bpc} B/cell) -> {achieved:.0f} GB/s")
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(cfg, kname, "float" if word == 4 else "double", tuning),
                           "kernel": f"{kname} level 0 ({cells} cells, {bpc} B/cell, {ms * 1e3:.2f} us/launch)"}
        out["vcycle"] = vcycle_bandwidth(fld, plan, stream, max(20, args.profile_reps // 10))
    return out, plan, E, K, st_


def vcycle_bandwidth(fld, plan, stream, reps):
    """Effective bandwidth of a whole outer iteration and of its multigrid V-cycle: the
    algorithmic bytes of every kernel of the pass (fld_plan_cycle_bytes) over the pass's
    mean time (HIP events on the bench stream, the iteration replayed from its graph)."""
    out = {}
    for name, what, kid in (("iteration", fld.FLD_CYCLE_ITERATION, fld.FLD_KERNEL_VCYCLE),
                            ("multigrid", fld.FLD_CYCLE_MG, fld.FLD_KERNEL_MG)):
        nbytes, launches = plan.cycle_bytes(what)
        ms, _ = plan.profile(kid, 0, reps, stream)
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"bytes": nbytes, "launches": launches, "us": ms * 1e3, "achieved_GBps": gbs,
                     "frac": gbs / HBM_PEAK_GBS}
        log(f"bench: {name}: {nbytes / 1e6:.1f} MB in {ms * 1e3:.1f} us ({launches} launches) -> {gbs:.0f} GB/s")
    return out


def mixed_vs_fp64_steps(fld, torch, grids, dev, nsteps: int, autotune: int):
    """The 256^3 step sequence in both precisions from the seeded input, untimed: per step the
    device's rel. residual, its residual under the oracle's operator and the error bound
    against the oracle's step it gives, and the mixed result's distance from the FP64 GPU
    result of the same step (each precision follows its own trajectory)."""
    g = grids[0]
    res = {}
    outs = {}
    for name, prec in (("fp64", fld.FLD_PREC_FP64), ("mixed", fld.FLD_PREC_MIXED)):
        plan = fld.Plan([g.E.shape], h=[g.h], precision=prec, rtol=1e-10, c=g.c, autotune=autotune)
        E = torch.from_numpy(np.ascontiguousarray(g.E)).to(dev)
        K = torch.from_numpy(np.ascontiguousarray(g.kappa_rho)).to(dev)
        out = torch.empty_like(E)
        steps = []
        outs[name] = []
        for k in range(nsteps):
            E_n = E.cpu().numpy()
            rc, (st,) = plan.step([E], [K], [out], [g.dt], check=False)
            torch.cuda.synchronize()
            x = out.cpu().numpy()
            rel, bound = certified_error(g, E_n, x)
            steps.append({"step": k, "cycles": int(st["cycles"]), "device_rel_residual": st["rel_residual"],
                          "oracle_operator_rel_residual": rel, "error_vs_fp64_oracle_bound": bound})
            outs[name].append(x if k == 0 else None)
            E.copy_(out)
            log(f"bench c3 {name} step {k}: cycles {st['cycles']} res {rel:.3e} error bound {bound:.3e}")
        res[name] = steps
        plan.close()
    x64, x32 = outs["fp64"][0], outs["mixed"][0]
    res["first_step_mixed_vs_fp64_gpu_rel_l2"] = float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64))
    return res


def main():
    args = parse()
    if args.config == "c5" and args.gpus == 1:
        serve_stream(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs one GPU's share of the work; --gpus must be 1"}))
        log("bench.py: only single-GPU runs are supported (the workload is one GPU's share)")
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2104_03968_amd as fld

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = args.config
    prec = args.precision or "fp64"
    precision = fld.FLD_PREC_MIXED if prec == "mixed" else fld.FLD_PREC_FP64
    log(f"bench: building inputs for {cfg} ({prec})")
    grids, has_gas, workload = build_config(W, cfg)
    ncells = sum(g.E.size for g in grids)

    m, plan, E, K, st_ = run_timed(fld, torch, args, cfg, grids, has_gas, precision, dev, args.steps, args.warmup)
    tuning = m["tuning"]
    out = {
        "metric": "cell-updates/s of implicit FLD step at 1e-10 residual; p50/p99 solve latency",
        "value": m["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == fld.FLD_PREC_FP64 else "f32-in-f64",
        "data": "synthetic",
        "config": {"workload": workload + (", fp64" if prec == "fp64" else ", FP32 V-cycles in FP64 defect correction"),
                   "cells": ncells, "grids": len(grids), "precision": prec,
                   "rtol": 1e-10, "fmg": plan.opts.fmg, "fmg_depths": plan.opts.fmg_depths, "coarse_op": args.coarse_op,
                   "krylov": plan.opts.krylov, "nu": [plan.opts.nu1, plan.opts.nu2], "nu_coarse": plan.opts.nu_coarse,
                   "launch": {k: tuning[k] for k in ("tile_rows", "tile_wide", "max_blocks", "tile_depth",
                                                     "fused3_levels", "tile_rows_coarse", "tile_rows_up",
                                                     "source")}},
        "step_latency_ms": m["latency_ms"],
        "vcycles_per_step": m["vcycles_per_step"],
        "roofline": m["roofline"],
        "vcycle_bandwidth": m["vcycle"],
    }
    if not args.no_extras:
        out["radiation_moments"] = time_moments(fld, plan, grids, E, K, torch.cuda.current_stream())
        if has_gas:
            log("bench: timing the IMEX step (tiring + exchange + implicit diffusion)")
            out["imex_step"] = time_imex(fld, plan, grids, E, st_["eps"], st_["rho"], st_["kap"], st_["gas"],
                                         torch.cuda.current_stream())
    plan.close()
    del E, K, st_
    if not args.no_extras:
        extra = {}
        if cfg in ("c3", "c4"):
            other = fld.FLD_PREC_MIXED if precision == fld.FLD_PREC_FP64 else fld.FLD_PREC_FP64
            mo, p2, *_ = run_timed(fld, torch, args, cfg, grids, has_gas, other, dev, args.steps, args.warmup)
            p2.close()
            key = "mixed" if other == fld.FLD_PREC_MIXED else "fp64"
            mo.pop("tuning")
            mo["speedup_vs_fp64"] = (mo["value"] / m["value"]) if key == "mixed" else (m["value"] / mo["value"])
            extra[key] = mo
        if cfg == "c3":
            extra["per_step_error_vs_fp64_oracle"] = mixed_vs_fp64_steps(fld, torch, grids, dev, 5, args.autotune)
        if cfg != "c2":
            g2, gas2, _ = build_config(W, "c2")
            m2, p3, *_ = run_timed(fld, torch, args, "c2", g2, gas2, fld.FLD_PREC_FP64, dev, args.steps, args.warmup)
            p3.close()
            m2.pop("tuning")
            extra["c2_1024sq_fp64_with_exchange"] = m2
        out["extra"] = extra
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline(W, cfg, grids, has_gas)
    print(json.dumps(out), flush=True)


def run_cpu_baseline(W, cfg, grids, has_gas):
    """The FP64 oracle on a bounded sample of the workload, on this host's cores."""
    if cfg == "c4":
        g0 = grids[0]
        sample = f"one FLD step of the first grid of the batch ({g0.E.shape[0]}^2)"
    else:
        g0 = grids[0]
        sample = f"one FLD step of the {'x'.join(map(str, g0.E.shape))} grid" + (" with exchange" if has_gas else "")
    log(f"bench: timing the FP64 CPU oracle: {sample}")
    t, info = cpu_baseline(g0, has_gas)
    return {"value": g0.E.size / t, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}; {info.method}, {info.iterations} iterations, {t:.1f} s; scipy sparse + numpy "
                      "(sparse matrix-vector products single-threaded)",
            "host": host_info(1)}


if __name__ == "__main__":
    main()
