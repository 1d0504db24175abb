"""Benchmark: cell-updates per second per pseudo-time stage of the dual-time Godunov solver.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload obstacle_dam_break]
                    [--precision f64] [--tile autotune|0x0|-WxL|TXxTY] [--unbatched]
                    [--cpu-budget S] [--no-mixed] [--no-extra]

A step is one real-time step (Algorithm 1): level n <- state, then pseudo-iterations of
s_max Runge-Kutta stages until the RMS residual is below the workload's tolerance or the
iteration cap is reached.  The default workload is the largest single-GPU configuration, the
4096 x 4096 dam break with a rectangular obstacle (4 x 4 walled tank, water at x < 1, y < 2,
solid cells at 2.5 < x < 2.7, y < 0.3, density ratio 1000:1, beta = 1100, dt = 2e-5, exactly 50
pseudo-iterations per step) in FP64, synthetic initial data; its planes (about 2 GB) exceed the
256 MB last-level cache, so the stage kernel streams from HBM.  Other workloads: hydrostatic,
dam_break (512 x 256), rayleigh_taylor, sloshing_ensemble (512 closed tanks starting at rest
with a tilted interface; its line carries a note on why).  The stage-kernel shape
comes from the library's autotuner (untimed, before the warmup).  The state stays resident in
HBM for the whole timed region; nothing crosses PCIe inside it except the per-step status read.

value = fluid cells x stages executed / seconds over exactly K timed steps (kernels replayed
from captured HIP graphs).  K defaults to the workload's own step count (200 for the obstacle
case), and the timed steps start from the initial state (it is set again after the W warmup
steps), so the timed region is the workload's whole run.  The roofline entry is the Runge-Kutta
stage kernel: algorithmic bytes per launch (per fluid cell-stage 109.3 B for FP64, the mean of
88 B at stage 1 and 120 B at later stages of a three-stage scheme; 74.7 B for the mixed form, 64
and 80 B) divided by its mean launch duration.  That duration is measured live inside the timed
region with HIP events on the library's stream: an event pair around every replayed graph of
pseudo-iterations, whose time divided by its stage launches is the mean (it includes the
dispatch gaps between the launches, the graph's one finalize launch and, with a tolerance, the
kernels of stopped tanks, which return at once; launches x mean <= the timed region).  traffic
is the copy-calibrated FETCH_SIZE + WRITE_SIZE bytes per
launch from the committed counter summaries in profiles/, reported only while the kernel
sources still hash to what was profiled.  valu is, from the same summaries, the stage kernel's
VALU instructions (SQ_INSTS_VALU x 64 lanes) per fluid cell-stage and their issue rate against
the chip's 39.3 T lane-instructions/s.  regime says whether the grid's planes exceed the 256 MB
last-level cache (below it, achieved is an effective rate, not HBM traffic).  stream_reference
sets the achieved rate beside the best rate of a plain plane-stream kernel of the library on the
same device (the FP64 stage's 11 planes in, 4 out, and a copy).  cpu_baseline times the serial
FP64 oracle on a bounded sample of the same workload (for the 4096^2 case a 2048 x 512 window of
the tank with the dam front and the obstacle), cpu_baseline_all_cores the same source built with
-fopenmp on all the host's threads.  An FP64 line also reports mixed_form: the mixed-precision
form on the same workload and steps, timed the same way after the FP64 measurement, with its
speedup (--no-mixed skips it).  The default line also carries extra_workloads: the 512 x 256 dam
break (cache-resident) in both forms, K of its steps (--no-extra skips it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
LLC_BYTES = 256e6              # MI355X last-level (Infinity) cache
# VALU issue ceiling: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 instruction takes 4 cycles;
# FP64 FMA issues at this rate, and so does unpacked FP32)
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
# bytes per cell of the grid's planes: three state buffers, level n, the flag byte (each further
# BDF level adds 32)
PLANE_BYTES = {"f64": 3 * 32 + 32 + 1, "mixed": 3 * 16 + 32 + 1}
BYTES_PER_CELL_STAGE = {       # algorithmic bytes per fluid cell per stage, three-stage mean
    "f64": (88.0 + 120.0 + 120.0) / 3.0,      # Q^{s-1} 32 + Q^0 32 + level n 24 + out 32
    "mixed": (64.0 + 80.0 + 80.0) / 3.0,      # deviations 16 + 16, level n 32, out 16
}


def kernel_source_hash() -> str:
    """Hash of the HIP/C++ sources of the library (the kernels a profile was taken of, and the
    host code that launches them; the plane-stream reference kernel is left out)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2108_08769_amd", "csrc", "*"))):
        if os.path.basename(f) == "stream_probe.hip":
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled(kind: str, workload: str, precision: str, tile: str):
    """A per-launch figure of the stage kernel from the committed counter summaries
    (profiles/*.md): kind "traffic" gives HBM bytes (copy-calibrated FETCH_SIZE + WRITE_SIZE),
    kind "valu" wave-level VALU instructions (SQ_INSTS_VALU).  None if no summary covers this
    workload, precision and tile, or the kernel sources changed since it was taken."""
    import glob
    src = kernel_source_hash()
    field = {"traffic": "bytes_per_launch", "valu": "insts_per_launch"}[kind]
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                if not line.startswith(kind + ":"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if (kv.get("workload") == workload and kv.get("precision") == precision
                        and kv.get("tile") == tile and kv.get("source") == src):
                    return float(kv[field])
    return None


def build_workload(name: str, precision: str):
    from paper_2108_08769_amd import workloads as wl
    if name == "dam_break":
        return wl.dam_break(precision=precision)
    if name == "hydrostatic":
        return wl.hydrostatic()
    if name == "rayleigh_taylor":
        return wl.rayleigh_taylor(precision=precision)
    if name == "obstacle_dam_break":
        return wl.obstacle_dam_break(precision=precision)
    if name == "sloshing_ensemble":
        return wl.sloshing_ensemble(precision=precision)
    raise SystemExit(f"unknown workload {name}")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The CPU baseline's sample of the 4096^2 obstacle case: columns 896..2943 and rows 0..511 of the
# tank (the dam front at x = 1, the obstacle at 2.5 < x < 2.7, y < 0.3), walls around the window.
# One oracle pseudo-iteration of the whole tank takes about 20 s on one core; the window's takes
# about 1.3 s, with the same work per cell.
CPU_WINDOW = {"obstacle_dam_break_4096x4096": (896, 2944, 0, 512)}


def sample_tank(wk):
    """The tank the CPU baseline times: the first tank (the only one, except in the ensemble), or
    its window for the 4096^2 case; and a phrase saying which."""
    import numpy as np
    from paper_2108_08769_amd import workloads as wl
    t = wk.tanks[0]
    if wk.name in CPU_WINDOW:
        i0, i1, j0, j1 = CPU_WINDOW[wk.name]
        dx, dy = t.lx / t.nx, t.ly / t.ny
        solid = None if t.solid is None else np.ascontiguousarray(t.solid[j0:j1, i0:i1])
        w = wl.Tank(i1 - i0, j1 - j0, (i1 - i0) * dx, (j1 - j0) * dy,
                    np.ascontiguousarray(t.q[:, j0:j1, i0:i1]), gx=t.gx, gy=t.gy, beta=t.beta,
                    bc=t.bc, solid=solid)
        return w, (f" (a {w.nx}x{w.ny} window of the tank: columns {i0}..{i1 - 1}, rows "
                   f"{j0}..{j1 - 1}, walls around it)")
    return t, (f" (its first tank, {t.nx}x{t.ny})" if len(wk.tanks) > 1 else "")


def cpu_baseline(wk, budget_s: float, omp: bool = False):
    """The oracle (FP64 C) timed on a bounded sample of the workload: real steps from the initial
    state of its sample tank (sample_tank), each with as many pseudo-iterations as the budget
    allows (up to the workload's cap), until the budget is used.  omp=False is the oracle as it
    stands (serial); omp=True the same source built with -fopenmp on all host threads (same
    results)."""
    import oracle
    t, what = sample_tank(wk)
    pb = oracle.Problem(t.nx, t.ny, t.lx, t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc,
                        solid=t.solid, stages=wk.stages, alpha=wk.alpha, cfl=wk.cfl, k=wk.k,
                        local_dtau=wk.local_dtau, bdf=1)
    t0 = time.perf_counter()
    oracle.step(pb, t.q, wk.dt, 1, 0.0, omp=omp)
    one = time.perf_counter() - t0
    iters = int(max(1, min(wk.max_pseudo, budget_s / max(one, 1e-6))))
    q, total_it, steps = t.q, 0, 0
    t0 = time.perf_counter()
    while True:
        q, it, _, rc = oracle.step(pb, q, wk.dt, iters, 0.0, omp=omp)
        total_it += it
        steps += 1
        spent = time.perf_counter() - t0
        if rc != 0 or spent + spent / steps > budget_s:  # the next step would not fit the budget
            break
    dt = time.perf_counter() - t0
    cell_stages = t.fluid_cells * wk.stages * total_it
    threads = oracle.threads(omp)
    return {"value": cell_stages / dt, "unit": "cell-updates/s per pseudo-time stage",
            "cores": threads, "kind": "oracle" if not omp else "oracle, -fopenmp build of the same source",
            "cpu": cpu_model(), "host_threads": os.cpu_count(),
            "sample": f"{wk.name}{what}: {steps} real step(s) of {iters} pseudo-iterations x "
                      f"{wk.stages} stages ({cell_stages:.3g} cell-stages, {dt:.1f} s, "
                      f"{threads} thread(s))"}


def measure(vdac, np, torch, wk, args, tune, tile, flux, pgrad, timing=True):
    """Warm-up, then the timed region of exactly args.steps real steps of wk (with timing, the
    stage-kernel events inside it give the roofline); returns the rate and what the JSON line
    reports."""
    tanks = [dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc,
                  solid=t.solid) for t in wk.tanks]
    opts = vdac.make_options(precision=wk.precision, stages=wk.stages, alpha=wk.alpha, cfl=wk.cfl,
                             k=wk.k, bdf=wk.bdf, tile=tile, graph_iters=args.graph_iters,
                             flux=flux, pgrad=pgrad, pk=args.pk, local_dtau=wk.local_dtau,
                             persistent=args.persistent)
    if tune and not args.unbatched:
        # untimed: the tuner times each candidate shape on scratch grids of the same tanks
        opts = vdac.autotune(tanks, opts, iters=5)
    chosen = f"{opts.tile_x}x{opts.tile_y}"
    if args.unbatched:
        grids = [vdac.Grid([td], opts) for td in tanks]
        for g, t in zip(grids, wk.tanks):
            g.set_state(0, t.q)
    else:
        grids = [vdac.Grid(tanks, opts)]
        for i, t in enumerate(wk.tanks):
            grids[0].set_state(i, t.q)
    fluid_per_grid = [np.array([t.fluid_cells for t in wk.tanks], dtype=np.float64)] \
        if not args.unbatched else [np.array([t.fluid_cells], dtype=np.float64) for t in wk.tanks]

    def step_all():
        iters, cs = 0, 0.0
        for g, fl in zip(grids, fluid_per_grid):
            _, done = g.step(wk.dt, wk.max_pseudo, wk.tol)
            iters += int(done.sum())
            cs += float((fl * done).sum()) * wk.stages
        return iters, cs

    for _ in range(args.warmup):
        step_all()
    # back to the initial state (outside the timed region), so that the timed steps are the
    # workload's own run from its start
    for g, tl in zip(grids, [[t] for t in wk.tanks] if args.unbatched else [wk.tanks]):
        for i, t in enumerate(tl):
            g.set_state(i, t.q)
    torch.cuda.synchronize()

    # timed region: exactly K steps, kernels replayed from captured graphs, with an event pair
    # around each replayed graph on the library's stream (the stage-kernel time)
    if timing:
        for g in grids:
            g.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    cell_stages = 0.0
    for _ in range(args.steps):
        it, cs = step_all()
        iters += it
        cell_stages += cs
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    roofline = None
    if timing:
        kms, launches, kcs = 0.0, 0, 0.0
        for g in grids:
            a, b, c = g.stage_timing_read()
            kms, launches, kcs = kms + a, launches + b, kcs + c
            g.stage_timing(False)
        if launches > 0 and kms > 0:
            bpc = BYTES_PER_CELL_STAGE[wk.precision] + 24.0 * (wk.bdf - 1)  # levels n-1, n-2
            avg_s = kms / 1e3 / launches
            bytes_per_launch = bpc * kcs / launches
            achieved = bytes_per_launch / avg_s / 1e9
            traffic = profiled("traffic", wk.name, wk.precision, chosen)
            valu = profiled("valu", wk.name, wk.precision, chosen)
            cells = kcs / launches
            grid_cells = sum(t.nx * t.ny for t in wk.tanks)
            plane_bytes = grid_cells * (PLANE_BYTES[wk.precision] + 32 * (wk.bdf - 1))
            resident = plane_bytes > LLC_BYTES
            roofline = {"bound": "hbm" if resident else "llc",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": None if traffic is None else int(round(traffic)),
                        "traffic_unit": "bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE)",
                        "traffic_vs_algorithmic": (None if traffic is None
                                                   else round(traffic / bytes_per_launch, 4)),
                        "kernel": "stage", "avg_launch_us": round(avg_s * 1e6, 3),
                        "launches": launches, "bytes_per_launch": bytes_per_launch,
                        "timed_ms_in_brackets": round(kms, 3),
                        "timed_region_ms": round(elapsed * 1e3, 3),
                        "regime": ("HBM-resident: the grid's planes (%.2f GB) exceed the 256 MB "
                                   "last-level cache" % (plane_bytes / 1e9) if resident else
                                   "cache-resident: the grid's planes (%.0f MB) fit the 256 MB "
                                   "last-level cache, so achieved is an effective rate (algorithmic "
                                   "bytes / launch time), not HBM traffic" % (plane_bytes / 1e6)),
                        "valu": None if valu is None else {
                            "insts_per_cell_stage": round(valu * 64 / cells, 1),
                            "achieved": round(valu * 64 / avg_s / 1e12, 2),
                            "peak": VALU_PEAK_T, "unit": "T lane-instructions/s",
                            "frac": round(valu * 64 / avg_s / 1e12 / VALU_PEAK_T, 4),
                            "source": "SQ_INSTS_VALU per launch (profiles/)"}}
    for g in grids:
        g.close()
    return {"value": cell_stages / elapsed, "elapsed": elapsed, "iters": iters, "chosen": chosen,
            "roofline": roofline}


def stream_reference(vdac, torch, n=16 << 20, reps=5, march=None):
    """Best rate, GB/s read + write, of the library's plane-stream kernel over three launch
    shapes: 11 FP64 planes of n cells read and 4 written (the FP64 stage's mix), and a plain
    copy of 4n doubles; 1.9 GB and 1 GB touched, well beyond the 256 MB last-level cache.
    march = (nx, ny, chunk): also the same plane mix in the row-marching stage kernel's access
    pattern on that tank (include/vdac_probe.h), as algorithmic GB/s (120 B per cell)."""
    inp = torch.zeros(11 * n, dtype=torch.float64, device="cuda")
    out = torch.empty(4 * n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    if march is not None and march[0] * march[1] <= n:
        nx, ny, chunk = march
        launch = lambda: vdac.march_probe(nx, ny, chunk, inp.data_ptr(), out.data_ptr(),
                                          stream.cuda_stream)
        launch()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            launch()
        e1.record(stream)
        e1.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        res["march_gbps"] = round(120.0 * nx * ny / sec / 1e9, 1)
    for n_in, n_out, cells, name in [(11, 4, n, "gbps"), (1, 1, 4 * n, "copy_gbps")]:
        best = 0.0
        for blocks in (0, 1024, 4096):
            launch = lambda: vdac.stream_probe(n_in, n_out, cells, blocks, inp.data_ptr(),
                                               out.data_ptr(), stream.cuda_stream)
            launch()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                launch()
            e1.record(stream)
            e1.synchronize()
            sec = e0.elapsed_time(e1) / 1e3 / reps
            best = max(best, (n_in + n_out) * 8.0 * cells / sec / 1e9)
        res[name] = round(best, 1)
    del inp, out
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed real steps (0: the workload's own step count, e.g. 500 for the "
                         "dam break)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="obstacle_dam_break")
    ap.add_argument("--precision", default="f64")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--tile", default="autotune",
                    help="stage kernel shape: autotune (the library's autotuner), 0x0 (built-in "
                         "heuristic), -WxL (row marching), or a 2D tile such as 3208x2")
    ap.add_argument("--max-pseudo", type=int, default=0,
                    help="override the workload's pseudo-iteration cap (short profiled runs)")
    ap.add_argument("--graph-iters", type=int, default=0,
                    help="pseudo-iterations per captured HIP graph (0 automatic, -1 no graphs)")
    ap.add_argument("--unbatched", action="store_true",
                    help="one grid per tank, stepped one after the other (the baseline of the "
                         "batched form)")
    ap.add_argument("--flux", default="osher", choices=["osher", "roe", "bassi"],
                    help="Riemann solver (Sec. 2.4)")
    ap.add_argument("--pgrad", default="new", choices=["new", "limiter", "split"],
                    help="pressure gradient (Sec. 2.3.2)")
    ap.add_argument("--pk", type=float, default=1.0, help="k of the limiter on p")
    ap.add_argument("--global-dtau", action="store_true", help="one pseudo-time step per tank")
    ap.add_argument("--bdf", type=int, default=0, help="BDF order (0: the workload's)")
    ap.add_argument("--persistent", action="store_true",
                    help="one persistent launch per stage (row-marching kernel)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run that an FP64 line reports beside it")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 512 x 256 dam break that the default line reports beside it")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only copy this many MiB device to device 20 times and print the rate "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this solver has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2108_08769_amd import vdac

    if args.copy_probe > 0:
        n = int(args.copy_probe * 2 ** 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"copy_probe_bytes_each_way": 4 * n, "copies": 20,
                          "GB_per_s_read_plus_write": 2 * 4 * n * 20 / dt / 1e9}), flush=True)
        return

    wk = build_workload(args.workload, args.precision)
    if args.steps <= 0:
        args.steps = wk.steps
    if args.max_pseudo > 0:
        wk.max_pseudo = args.max_pseudo
    if args.bdf > 0:
        wk.bdf = args.bdf
    if args.global_dtau:
        wk.local_dtau = False
    flux = {"osher": vdac.FLUX_OSHER, "roe": vdac.FLUX_ROE, "bassi": vdac.FLUX_BASSI}[args.flux]
    pgrad = {"new": vdac.PGRAD_NEW, "limiter": vdac.PGRAD_LIMITER, "split": vdac.PGRAD_SPLIT}[args.pgrad]
    torch.cuda.set_device(0)
    tune = args.tile == "autotune"
    tile = (0, 0) if tune else tuple(int(v) for v in args.tile.lower().split("x"))
    res = measure(vdac, np, torch, wk, args, tune, tile, flux, pgrad, timing=not args.no_stage_timing)
    value, elapsed, iters, chosen, roofline = (res[k] for k in ("value", "elapsed", "iters", "chosen",
                                                                  "roofline"))
    fluid = wk.fluid_cells

    line = {
        "metric": "cell-updates/s per pseudo-time stage",
        "value": value,
        "unit": "cell-updates/s per pseudo-time stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wk.precision == "f64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wk.name, "cells": fluid, "precision": wk.precision,
                   "tile": chosen + (" (autotuned)" if tune and not args.unbatched else ""),
                   "tanks": len(wk.tanks), "batched": not args.unbatched,
                   "graph_iters": args.graph_iters,
                   "dt": wk.dt, "max_pseudo": wk.max_pseudo, "tol": wk.tol,
                   "rk_stages": wk.stages, "pseudo_iterations": iters, "flux": args.flux,
                   "pgrad": args.pgrad, "local_dtau": bool(wk.local_dtau), "bdf": wk.bdf,
                   "persistent": bool(args.persistent)},
        "roofline": roofline,
    }
    if args.workload == "sloshing_ensemble":
        line["config"]["note"] = (
            "512 closed tanks that start at rest with a tilted interface; a uniform initial "
            "horizontal velocity in closed tanks makes the pseudo-time iteration diverge (the "
            "oracle's too), so the fourth draw per tank is the tilt")
    if roofline is not None:
        march = None
        if len(wk.tanks) == 1 and chosen.startswith("-"):
            march = (wk.tanks[0].nx, wk.tanks[0].ny, int(chosen.split("x")[1]))
        ref = stream_reference(vdac, torch, march=march)
        roofline["stream_reference"] = {
            "kernel": "plane stream: 11 FP64 planes read, 4 written, one cell per lane "
                      "(include/vdac_probe.h)",
            "gbps": ref["gbps"], "copy_gbps": ref["copy_gbps"],
            "frac": round(roofline["achieved"] / ref["gbps"], 4)}
        if "march_gbps" in ref:
            roofline["march_reference"] = {
                "kernel": "the same 11-in, 4-out plane mix in the stage kernel's row-marching "
                          "pattern on this tank and chunk, no arithmetic (include/vdac_probe.h); "
                          "algorithmic GB/s at 120 B per cell",
                "gbps": ref["march_gbps"],
                "frac": round(roofline["achieved"] / ref["march_gbps"], 4)}
    # the mixed form on the same workload, after the FP64 line's measurement (reported beside
    # it: the headline metric compares the two forms)
    if wk.precision == "f64" and not args.no_mixed:
        wkm = build_workload(args.workload, "mixed")
        if wkm.precision == "mixed":
            if args.max_pseudo > 0:
                wkm.max_pseudo = args.max_pseudo
            if args.bdf > 0:
                wkm.bdf = args.bdf
            if args.global_dtau:
                wkm.local_dtau = False
            rm = measure(vdac, np, torch, wkm, args, tune, tile, flux, pgrad,
                         timing=not args.no_stage_timing)
            line["mixed_form"] = {"value": rm["value"], "unit": line["unit"],
                                  "ms_per_step": rm["elapsed"] * 1e3 / args.steps,
                                  "speedup_vs_f64": rm["value"] / value, "dtype": "f32+f64",
                                  "tile": rm["chosen"] + (" (autotuned)" if tune and not args.unbatched else ""),
                                  "pseudo_iterations": rm["iters"],
                                  "note": "same workload, steps and timing; FP32 storage as deviations "
                                          "from FP64 level n, FP32 reconstruction and fluxes, FP64 "
                                          "residual, sources and update",
                                  "roofline": rm["roofline"]}
    # the cache-resident 512 x 256 dam break beside the default workload (both forms, K steps)
    if args.workload == "obstacle_dam_break" and not args.no_extra and not args.unbatched:
        extra = {}
        for prec in ("f64", "mixed"):
            wke = build_workload("dam_break", prec)
            re_ = measure(vdac, np, torch, wke, args, tune, (0, 0) if tune else tile, flux, pgrad,
                          timing=False)
            extra[prec] = {"value": re_["value"], "ms_per_step": re_["elapsed"] * 1e3 / args.steps,
                           "tile": re_["chosen"] + (" (autotuned)" if tune else ""),
                           "pseudo_iterations": re_["iters"]}
        extra["f64"]["unit"] = line["unit"]
        extra["mixed_speedup_vs_f64"] = extra["mixed"]["value"] / extra["f64"]["value"]
        extra["note"] = ("dam break 512 x 256 (water x < 1, y < 1 in a 4 x 2 tank, dt = 1e-4, up "
                         "to 100 pseudo-iterations to 1e-6), its first K steps; cache-resident")
        line["extra_workloads"] = {wke.name: extra}
    if args.cpu_budget > 0:
        line["cpu_baseline"] = cpu_baseline(wk, args.cpu_budget)
        line["cpu_baseline_all_cores"] = cpu_baseline(wk, args.cpu_budget, omp=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
