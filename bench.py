#!/usr/bin/env python3
"""Throughput of the DS-PHD/MIB particle recursion on one MI355X.

A step is one full filter cycle (predict, assign, update, moments, resample) of the 512x512 grid
at 0.2 m with 2^21 persistent and 2^18 new-born particles over a synthetic ray-cast scene
(30 moving boxes, 1 % static clutter).  Measurement grids are generated and uploaded before the
timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--cpu-seconds S] [--copy-calibration]
    python bench.py --traffic-from FETCH.csv WRITE.csv --traffic-command CMD ...

The timed region replays K cycles captured as HIP graphs (one graph per cycle, each with its own
measurement grid), so host launch overhead is out of the loop; the same K cycles stepped call by
call are timed before it and reported as `eager`.  The roofline object covers the kernel that
takes the most time per cycle (found from a traced warm-up): its launches in the eager cycles are
bracketed by HIP events on their own stream (event records captured inside a graph do not
bracket the kernel nodes on this stack), and its algorithmic bytes per launch (the
per-particle / per-cell figures below, times the units one launch processes) are divided by the
mean launch duration.  HBM traffic comes from the committed counter summary of
that kernel when its source has not changed since.

Two execution modes follow the headline run (`modes` in the JSON line): a batch of 16 grids of
mixed sizes stepped with one launch per kernel (against the same grids stepped one after
another), and 64 streams served with Poisson arrivals through the serving runtime (request
latency p50 / p99 at real time and at an accelerated replay).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "filter cycles/s and particles/s at 512²/2M; p50/p99 cycle latency multi-stream"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes of a whole cycle (each array read / written once per step that needs it,
# the sort as one ideal pass, random numbers in registers): per persistent particle, per
# new-born slot, per cell.
B_PER_PARTICLE = 156
B_PER_BORN = 28
B_PER_CELL = 92

CSRC = os.path.join(ROOT, "paper_1605_02406_amd", "csrc")
KERNEL_SOURCE = {
    "k_predict": "k_particles.hip", "k_sort_hist": "k_sort.hip", "k_scan_rows": "k_sort.hip",
    "k_sort_scatter": "k_sort.hip", "k_seg_sums<false>": "k_cells.hip", "k_scan_parts":
    "k_particles.hip",
    "k_seg_sums<true>": "k_cells.hip", "k_cells<false>": "k_cells.hip",
    "k_cells<true>": "k_cells.hip", "k_seg_moments": "k_cells.hip",
    "k_born_offsets": "k_particles.hip", "k_particle_tiles": "k_particles.hip",
    "k_resample": "k_resample.hip", "k_resample_windowed": "k_resample.hip",
}


def sort_plan(C: int, max_bits: int = 11, sort_passes: int = 0):
    """Digit widths of the radix sort of keys 0..C under a launch plan's sort_passes, as the
    library sets them: the fewest passes of at most max_bits bits, or more, evenly split."""
    kb = max(1, C.bit_length())
    passes = max((kb + max_bits - 1) // max_bits, sort_passes)
    bits, left = [], kb
    for q in range(passes):
        b = (left + (passes - q) - 1) // (passes - q)
        bits.append(b)
        left -= b
    return bits


def algorithmic_bytes(kernel: str, nu: int, nb: int, C: int, sort_passes: int = 0) -> float:
    """Algorithmic bytes of ONE launch of `kernel` on one grid (averaged over the launches of a
    cycle where they differ), from per-unit figures: predict reads x, y, vx, vy, w (20 B) and
    writes them and the key (24 B); the
    resampling reads every joint weight (4 B), the state of each chosen source (16 B) and
    writes the 20-byte state of every output; the per-cell pass of the assignment reads the
    sorted key, weight and velocity (16 B per particle) and writes the cell range and six FP64
    sums per cell (56 B); the cell pass reads ranges, sums, m_F and the measurement (68 B) and
    writes the weight sum, masses, normalisers and moments (73 B) per cell; the row scans read
    and write every entry of a digit histogram (one per digit and 4096-key tile); the slot
    offsets read rho_b and
    write o_c (8 B per cell); the tile pass rescales the persistent weights (key and weight
    read, weight written: 12 B per particle) and writes each new-born slot's 25-byte record.
    The sort counts as one ideal pass over the 24-byte record (read and written once: 48 B per
    particle and cycle), shared evenly by its scatter launches; the scan of the partial sums
    reads and writes one 8-byte sum per tile."""
    bits = sort_plan(C, sort_passes=sort_passes)
    if kernel == "k_predict":
        return 44.0 * nu
    if kernel == "k_sort_scatter":
        return 48.0 * nu / len(bits)
    if kernel == "k_scan_parts":
        return 16.0 * (-(-nu // 1024) + -(-nb // 256))
    if kernel == "k_sort_hist":
        return 4.0 * nu
    if kernel == "k_scan_rows":
        tiles = -(-nu // 4096)
        return 8.0 * sum(1 << b for b in bits) * tiles / len(bits)
    if kernel == "k_seg_sums<false>":
        return 16.0 * nu + 56.0 * C
    if kernel == "k_seg_sums<true>":
        return 16.0 * nu + 16.0 * C
    if kernel in ("k_cells<false>", "k_cells<true>"):
        return (68.0 + 73.0) * C
    if kernel in ("k_resample", "k_resample_windowed"):
        return 4.0 * (nu + nb) + 16.0 * nu + 20.0 * nu
    if kernel == "k_particle_tiles":
        return 12.0 * nu + 25.0 * nb
    if kernel == "k_born_offsets":
        return 8.0 * C
    return float("nan")


def source_digest(kernel: str) -> str:
    """SHA-256 of the kernel's source file and of the headers every kernel includes."""
    h = hashlib.sha256()
    for f in (KERNEL_SOURCE[kernel], "dogm_internal.h", "launch.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


PROFILES = os.path.join(ROOT, "profiles")


def traffic_path(workload: str, outdir: str = PROFILES) -> str:
    return os.path.join(outdir, f"traffic_{workload}.json")


def measured_traffic(kernel: str, workload: str, outdir: str = PROFILES):
    """HBM bytes per launch from the committed counter summary, or None if there is none or
    the kernel's source changed since the counters were taken."""
    path = traffic_path(workload, outdir)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get("kernels", {}).get(kernel)
    if not rec or rec.get("source_sha256") != source_digest(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def precision_study(path: str = os.path.join(PROFILES, "precision_c1024.json")):
    """The committed record of the precision study on the 1024x1024 workload (maximum and 99th
    percentile of each output's error against the oracle in both precision modes, and the
    resampling indices that plain FP64 and FP32 CDFs would change), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    keep = ("predict.x", "predict.vx", "update.m_O", "update.rho_b", "update.w", "born.x",
            "moments.mean_x", "moments.var_x")
    return {"workload": rec["workload"], "source": "profiles/precision_c1024.json",
            "modes": {m["mode"]: {"errors": {k: v for k, v in m["errors"].items() if k in keep},
                                  "resample_cdf_variants": {
                                      k: v["indices_differing"]
                                      for k, v in m["resample_cdf_variants"].items() if k != "W"}}
                      for m in rec["modes"]}}


def measured_copy_gbs(dev, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Bandwidth of a plain device-to-device copy of `nbytes` (bytes read + bytes written per
    second, median of `reps` event-timed copies): the practical HBM ceiling beside the vendor's
    8 TB/s."""
    import numpy as np
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / float(np.median(times)) / 1e9


def short_name(full: str) -> str:
    """Kernel name as the trace hook reports it, from the demangled name in a counter file."""
    name = full.split("(")[0].replace("void ", "").replace("dogm::", "").strip()
    # the precision mode's template argument is not part of the traced name
    for t in ("<float>", "<double>"):
        name = name.replace(t, "")
    return name.replace(", float>", ">").replace(", double>", ">")


def write_traffic(fetch_csv: str, write_csv: str, workload: str, commands, outdir: str = PROFILES):
    """Turns two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) into HBM
    bytes per launch of every kernel, calibrated by the same counters on the 1 GiB device copy
    that --copy-calibration runs, and writes the JSON record and a markdown table."""
    import csv

    def load(path, counter):
        per = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return per

    f = load(fetch_csv, "FETCH_SIZE")
    w = load(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    copy_f = max(f.get("__amd_rocclr_copyBuffer", [0.0]))
    copy_w = max(w.get("__amd_rocclr_copyBuffer", [0.0]))
    if copy_f <= 0 or copy_w <= 0:
        raise SystemExit("no 1 GiB calibration copy in the counter files (run with --copy-calibration)")
    ff, wf = gib_kib / copy_f, gib_kib / copy_w
    rec = {"workload": workload, "fetch_factor": ff, "write_factor": wf,
           "calibration": {"copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
                           "copy_bytes": 1 << 30},
           "commands": commands, "kernels": {}}
    lines = [f"# HBM traffic per kernel launch, {workload}", "", "Commands (two separate counter passes):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", f"Calibration: the 1 GiB device copy reads FETCH_SIZE = {copy_f:.0f} KiB and "
                  f"WRITE_SIZE = {copy_w:.0f} KiB, so bytes read = {ff:.3f} x FETCH_SIZE and "
                  f"bytes written = {wf:.3f} x WRITE_SIZE (KiB = 1024 B).", "",
              "Mean over the launches in the run; MB = 10^6 bytes after calibration; algorithmic "
              "bytes per launch as bench.py counts them.", "",
              "| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB | "
              "algorithmic MB | traffic / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    from paper_1605_02406_amd import scenes
    wl = scenes.WORKLOADS[workload]
    nu, nb, C = wl["n_pers"], wl["n_born"], wl["nx"] * wl["ny"]
    for full in sorted(f):
        name = short_name(full)
        if name not in KERNEL_SOURCE or full not in w:
            continue
        fk = sum(f[full]) / len(f[full])
        wk = sum(w[full]) / len(w[full])
        rd, wr = fk * 1024 * ff, wk * 1024 * wf
        alg = algorithmic_bytes(name, nu, nb, C)
        rec["kernels"][name] = {"launches": len(f[full]), "fetch_kib": fk, "write_kib": wk,
                                "read_bytes": rd, "written_bytes": wr,
                                "hbm_bytes_per_launch": rd + wr,
                                "algorithmic_bytes_per_launch": alg,
                                "source_sha256": source_digest(name)}
        lines.append(f"| `{name}` | {len(f[full])} | {fk:.0f} | {wk:.0f} | {rd / 1e6:.1f} | "
                     f"{wr / 1e6:.1f} | {alg / 1e6:.1f} | {(rd + wr) / alg:.2f} |")
    with open(traffic_path(workload, outdir), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    with open(os.path.join(outdir, f"hbm_traffic_{workload}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c512")
    ap.add_argument("--model", choices=("ds", "phd"), default="ds",
                    help="per-cell step: Dempster-Shafer (Sec. VI) or particle PHD/MIB (Sec. V)")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32",
                    help="FP32 state with exact integer decisions (default) or all-FP64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="host time budget of the oracle's CPU baseline: whole cycles are run "
                         "until it is spent (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 1 GiB (for counter calibration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's default launch plan instead of the autotuner's")
    ap.add_argument("--plan", default=None, metavar="P,S,R",
                    help="fixed launch plan sort_passes,scan_parts,resample (no tuning); "
                         "a profile of the tuned bench uses the plan the tuner printed")
    ap.add_argument("--closed-loop-steps", type=int, default=50,
                    help="timed cycles of the closed loop in which the device generates every "
                         "measurement grid from the moving scene (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="timed cycles of the 16-grid batch (0: skip the batched mode)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="simulated seconds of the 64-stream serving replay (0: skip serving)")
    ap.add_argument("--serve-realtime-seconds", type=float, default=10.0,
                    help="simulated seconds replayed at real time (speed 1), the rest of the "
                         "speeds replay --serve-seconds")
    ap.add_argument("--serve-speedups", default="1,10,30,100,300",
                    help="replay speeds of the serving run (1 = real time)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="HBM budget for admitting serving streams")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 counter files into the traffic record")
    ap.add_argument("--traffic-command", action="append", default=[],
                    help="command line recorded with --traffic-from (repeat for each pass)")
    return ap.parse_args()


def main():
    args = parse()
    if args.traffic_from:
        write_traffic(args.traffic_from[0], args.traffic_from[1], args.workload,
                      args.traffic_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU: the implementation has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1605_02406_amd import dogm, scenes

    wl = scenes.WORKLOADS[args.workload]
    p = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"],
                         seed=wl.get("seed", 0),
                         model=dogm.MODEL_PHD_MIB if args.model == "phd" else dogm.MODEL_DS,
                         precision=(dogm.PRECISION_FP64 if args.precision == "fp64"
                                    else dogm.PRECISION_FP32),
                         **scenes.FILTER)
    C = wl["nx"] * wl["ny"]
    nu, nb = wl["n_pers"], wl["n_born"]
    n_cycles = args.warmup + 2 * args.steps
    print(f"[bench] generating {n_cycles} measurement grids", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    seq = scenes.measurement_sequence(wl, n_cycles, model=args.model)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    meas = [dogm.Meas(**{k: torch.as_tensor(v, device=dev) for k, v in m.items()}) for m in seq]
    plan, tuning = None, None
    if args.plan:
        from paper_1605_02406_amd import tune
        ps, sp, rs = (int(x) for x in args.plan.split(","))
        plan = dict(sort_passes=ps, scan_parts=sp, resample=rs)
        p = tune.with_plan(p, plan)
    elif not args.no_tune:
        from paper_1605_02406_amd import tune
        print("[bench] tuning the launch plan", file=sys.stderr, flush=True)
        plan, tuning = tune.tune(p, meas=meas[:8])
        p = tune.with_plan(p, plan)
    g = dogm.Grid(p)
    torch.cuda.synchronize()

    # warm-up; its last cycles are traced kernel by kernel to find the dominant kernel
    print(f"[bench] warm-up {args.warmup} cycles", file=sys.stderr, flush=True)
    n_traced = min(3, args.warmup)
    for k in range(args.warmup - n_traced):
        g.step(meas[k])
    with dogm.KernelTrace(None, capacity=64 * max(n_traced, 1)) as tr:
        for k in range(args.warmup - n_traced, args.warmup):
            g.step(meas[k])
    torch.cuda.synchronize()
    per_kernel = {}
    for name, ms in zip(tr.names(), tr.durations_ms()):
        per_kernel.setdefault(name, []).append(ms)
    per_kernel_ms = {k: float(np.sum(v)) / max(n_traced, 1) for k, v in per_kernel.items()}
    launches = {k: len(v) // max(n_traced, 1) for k, v in per_kernel.items()}
    dominant = max(per_kernel_ms, key=per_kernel_ms.get) if per_kernel_ms else "k_predict"

    # eager reference: the calls of every step launched from the host, HIP events between the
    # calls on the grid's stream (the current stream)
    print(f"[bench] eager {args.steps} cycles", file=sys.stderr, flush=True)
    names = ["predict", "assign", "update", "moments", "resample"]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    dom = dogm.KernelTrace(dominant, capacity=args.steps * max(launches.get(dominant, 1), 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with dom:
        for s in range(args.steps):
            e = ev[s]
            m = meas[args.warmup + s]
            e[0].record()
            g.predict()
            e[1].record()
            g.assign()
            e[2].record()
            g.update(m)
            e[3].record()
            g.moments()
            e[4].record()
            g.resample()
            e[5].record()
        torch.cuda.synchronize()
    eager_wall = time.perf_counter() - t0

    # timed region: the next K cycles captured one graph per cycle, replayed back to back
    print(f"[bench] capturing {args.steps} cycles", file=sys.stderr, flush=True)
    side = torch.cuda.Stream()
    graphs = []
    for s in range(args.steps):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            g.step(meas[args.warmup + args.steps + s])
        graphs.append(gr)
    gev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    print(f"[bench] timing {args.steps} graph replays", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        gev[s][0].record()
        graphs[s].replay()
        gev[s][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = g.status()
    print("[bench] timed region done", file=sys.stderr, flush=True)
    # new-born mass of the last cycle that fell on cells whose share of the nu_b slots rounds to
    # none (no carrier): lost from the next cycle's state
    rho_b = g.v["rho_b"].double()
    off = g.v["born_off"].long()
    no_slot = (rho_b > 0) & (off[1:] == off[:-1])
    births_lost = {"cells_with_births": int((rho_b > 0).sum()),
                   "cells_without_slot": int(no_slot.sum()),
                   "mass_without_slot": float(rho_b[no_slot].sum()),
                   "fraction_of_new_born_mass": float(rho_b[no_slot].sum() / max(float(rho_b.sum()),
                                                                                   1e-300))}

    per_call = {n: float(np.mean([ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(args.steps)]))
                for i, n in enumerate(names)}
    eager_cycle_ms = [ev[s][0].elapsed_time(ev[s][5]) for s in range(args.steps)]
    cycle_ms = [gev[s][0].elapsed_time(gev[s][1]) for s in range(args.steps)]
    ms_per_step = wall * 1e3 / args.steps
    cycles_per_s = args.steps / wall
    bytes_cycle = b_alg(nu, nb, C)

    dom_ms = dom.durations_ms()
    dom_mean_ms = float(np.mean(dom_ms)) if dom_ms else float("nan")
    dom_bytes = algorithmic_bytes(dominant, nu, nb, C, sort_passes=p.sort_passes)
    dom_gbs = dom_bytes / (dom_mean_ms * 1e-3) / 1e9
    traffic = measured_traffic(dominant, args.workload)

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    copy_gbs = measured_copy_gbs(dev)
    # a copy whose 2 x 48 MB stay in the 256 MB last-level cache, the size of one cycle's arrays
    copy_cached_gbs = measured_copy_gbs(dev, nbytes=48 << 20, reps=50)

    out = {
        "metric": METRIC,
        "value": cycles_per_s,
        "unit": "cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": describe_workload(wl) + (
                       "; particle PHD/MIB model (Sec. V)" if args.model == "phd" else "") + (
                       "; all-FP64 precision mode" if args.precision == "fp64" else ""),
                   "nx": wl["nx"], "ny": wl["ny"], "cell_m": wl["cell"], "n_pers": nu,
                   "n_born": nb},
        "particles_per_s": cycles_per_s * nu,
        "all_particles_per_s": cycles_per_s * (nu + nb),
        "cycle_ms_p50": float(np.percentile(cycle_ms, 50)),
        "cycle_ms_p99": float(np.percentile(cycle_ms, 99)),
        "eager": {"ms_per_step": eager_wall * 1e3 / args.steps,
                  "cycles_per_s": args.steps / eager_wall,
                  "cycle_ms_p50": float(np.percentile(eager_cycle_ms, 50)),
                  "cycle_ms_p99": float(np.percentile(eager_cycle_ms, 99)),
                  "per_call_ms": per_call},
        "per_kernel_ms": per_kernel_ms,
        "launches_per_cycle": launches,
        "cycle_roofline": {"bound": "hbm", "algorithmic_bytes": bytes_cycle,
                           "achieved": bytes_cycle / (ms_per_step * 1e-3) / 1e9,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": bytes_cycle / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "frac_of_measured_copy":
                               bytes_cycle / (ms_per_step * 1e-3) / 1e9 / copy_gbs},
        "roofline": {"kernel": dominant, "bound": "hbm", "achieved": dom_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": dom_bytes,
                     "launch_ms_mean": dom_mean_ms, "launches_timed": len(dom_ms),
                     "measured_copy_GBps": copy_gbs, "frac_of_measured_copy": dom_gbs / copy_gbs,
                     "measured_copy_cache_resident_GBps": copy_cached_gbs},
        "status_word": status,
        "launch_plan": {"plan": plan, "tuning_ms_per_cycle": tuning},
        "births_without_slot": births_lost,
        "meas_generation_s": t_gen,
        # the assignment (radix sort and per-cell pass) against one ideal pass that reads and
        # writes a 24-byte record once: 8 TB/s / 48 B
        "sort": {"keys_per_s": nu / (per_call["assign"] * 1e-3),
                 "ideal_pass_keys_per_s": HBM_PEAK_GBS * 1e9 / 48.0},
    }

    study = precision_study()
    if study is not None:
        out["precision_study"] = study

    modes = {}
    if args.closed_loop_steps > 0:
        print("[bench] closed loop: device sensor + filter", file=sys.stderr, flush=True)
        modes["closed_loop_device_sensor"] = bench_closed_loop(wl, p, args.closed_loop_steps)
    if args.batch_steps > 0:
        print("[bench] batched mode: 16 grids", file=sys.stderr, flush=True)
        modes["batched_16_grids"] = bench_batched(args.batch_steps, tuned=not args.no_tune)
    if args.serve_seconds > 0:
        print("[bench] serving mode: 64 streams", file=sys.stderr, flush=True)
        modes["served_64_streams"] = bench_served(
            args.serve_seconds, [float(x) for x in args.serve_speedups.split(",") if x],
            int(args.serve_budget_gib * (1 << 30)), realtime_seconds=args.serve_realtime_seconds)
    if modes:
        out["modes"] = modes

    if args.cpu_seconds > 0:
        print(f"[bench] oracle on the host, {args.cpu_seconds:.0f} s", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, seq, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def _pow2(n: int) -> str:
    return f"2^{n.bit_length() - 1}" if n > 0 and n & (n - 1) == 0 else str(n)


def describe_workload(wl: dict) -> str:
    scene = (f"ray-cast scene of {wl['n_boxes']} moving boxes + {wl['clutter'] * 100:g}% clutter"
             if wl["scene"] == "boxes" else "ray-cast scene of 3 moving boxes and 2 walls")
    return (f"{wl['nx']}x{wl['ny']} grid at {wl['cell']:g} m, {_pow2(wl['n_pers'])} persistent + "
            f"{_pow2(wl['n_born'])} new-born particles, {scene}")


def b_alg(nu: int, nb: int, C: int) -> int:
    return B_PER_PARTICLE * nu + B_PER_BORN * nb + B_PER_CELL * C


def bench_closed_loop(wl: dict, p, steps: int, warmup: int = 5):
    """The scene, the sensor and the filter in one loop on the device: per cycle the truth grid
    of the moving scene (dogm_sensor_truth), the ray cast and detections (dogm_sensor_scan) and
    the filter cycle, captured as one HIP graph per cycle and replayed.  Only the boxes'
    rectangles come from the host, uploaded for every cycle before the timed region."""
    import numpy as np
    import torch

    from paper_1605_02406_amd import dogm, scenes

    dev = torch.device("cuda:0")
    n = warmup + steps
    sc = scenes.make_scene(wl, wl.get("seed", 0))
    rects = []
    for _ in range(n):
        sc.advance()
        rects.append(sc.rects())
    rects = torch.as_tensor(np.stack(rects), dtype=torch.float64, device=dev)
    static = torch.as_tensor(sc.static_mask().reshape(-1).astype(np.uint8), device=dev)
    C = sc.nx * sc.ny
    occ = torch.zeros(C, dtype=torch.uint8, device=dev)
    seen = torch.zeros_like(occ)
    m_occ = torch.zeros(C, dtype=torch.float32, device=dev)
    m_free = torch.zeros_like(m_occ)
    meas = dogm.Meas(m_occ, m_free)
    g = dogm.Grid(p)

    def cycle(k, stream=None):
        dogm.sensor_truth(rects[k], static, sc.nx, sc.ny, sc.cell, occ, stream=stream)
        dogm.sensor_scan(occ, sc.nx, sc.ny, scenes.SENSOR["p_d"], scenes.SENSOR["p_cl"], 4242,
                         k + 1, seen, m_occ, m_free, stream=stream)
        g.step(meas)

    for k in range(warmup):
        cycle(k)
    side = torch.cuda.Stream()
    graphs = []
    for k in range(warmup, n):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            cycle(k, stream=side)
        graphs.append(gr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gr in graphs:
        gr.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    with dogm.KernelTrace(None, capacity=64) as tr:
        cycle(warmup)  # one more eager cycle, traced, for the sensor's share
    torch.cuda.synchronize()
    sensor_ms = sum(d for nm, d in zip(tr.names(), tr.durations_ms()) if nm.startswith("k_sensor"))
    return {"steps": steps, "ms_per_cycle": wall * 1e3 / steps, "cycles_per_s": steps / wall,
            "sensor_kernels_ms_per_cycle": sensor_ms, "observed_cells_last_cycle":
            int(seen.sum().item()), "status_word": g.status()}


def bench_batched(steps: int, warmup: int = 5, tuned: bool = True):
    """16 grids of mixed sizes (4x128^2, 4x256^2, 3x384^2, 3x512^2, 2x768^2, 8 particles and one
    new-born slot per cell) stepped together, one launch per kernel for the whole batch, each
    batched cycle captured as a HIP graph and replayed; then the same grids stepped one after
    another (the plain per-grid loop), captured and replayed alike.  With `tuned`, every grid
    shape's launch plan comes from the autotuner (the same plans in both modes)."""
    import numpy as np
    import torch

    from paper_1605_02406_amd import dogm, scenes

    dev = torch.device("cuda:0")
    wls = [scenes.batch_workload(n, seed=i) for i, n in enumerate(scenes.BATCH_SIZES)]
    n_cycles = warmup + 2 * steps
    seqs = []
    for wl in wls:
        seqs.append([dogm.Meas(torch.as_tensor(m["m_occ"], device=dev),
                               torch.as_tensor(m["m_free"], device=dev))
                     for m in scenes.measurement_sequence(wl, n_cycles)])
    params = [dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"],
                               seed=i, grid_id=i, **scenes.FILTER) for i, wl in enumerate(wls)]
    plans = {}
    if tuned:
        from paper_1605_02406_amd import tune
        for i, prm in enumerate(params):
            plan, rep = tune.tune(prm)
            plans[f'{prm.nx}x{prm.ny}'] = {"plan": plan, "tuning_ms_per_cycle": rep}
            params[i] = tune.with_plan(prm, plan)
    grids = [dogm.Grid(prm) for prm in params]
    for k in range(warmup):
        dogm.step_batch(grids, [sq[k] for sq in seqs])
    torch.cuda.synchronize()

    def replay(graphs):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in graphs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e, gr in zip(ev, graphs):
            e[0].record()
            gr.replay()
            e[1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, [e[0].elapsed_time(e[1]) for e in ev]

    side = torch.cuda.Stream()
    batched = []
    for s in range(steps):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            dogm.step_batch(grids, [sq[warmup + s] for sq in seqs])
        batched.append(gr)
    wall_b, ms_b = replay(batched)
    looped = []
    for s in range(steps):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            for g, sq in zip(grids, seqs):
                g.step(sq[warmup + steps + s])
        looped.append(gr)
    wall_l, ms_l = replay(looped)
    status = [g.status() for g in grids]
    nu = sum(wl["n_pers"] for wl in wls)
    nb = sum(wl["n_born"] for wl in wls)
    C = sum(wl["nx"] * wl["ny"] for wl in wls)
    bytes_cycle = sum(b_alg(wl["n_pers"], wl["n_born"], wl["nx"] * wl["ny"]) for wl in wls)
    ms = wall_b * 1e3 / steps
    return {"grids": [f'{wl["nx"]}x{wl["ny"]}' for wl in wls], "cells": C, "n_pers": nu,
            "n_born": nb, "steps": steps, "warmup": warmup,
            "batched": {"ms_per_cycle": ms, "cycles_per_s": 1e3 / ms,
                        "grid_cycles_per_s": len(wls) * 1e3 / ms,
                        "particles_per_s": nu * 1e3 / ms,
                        "cycle_ms_p50": float(np.percentile(ms_b, 50)),
                        "cycle_ms_p99": float(np.percentile(ms_b, 99)),
                        "roofline_frac": bytes_cycle / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "per_grid_loop": {"ms_per_cycle": wall_l * 1e3 / steps,
                              "cycles_per_s": steps / wall_l,
                              "particles_per_s": nu * steps / wall_l},
            "algorithmic_bytes_per_cycle": bytes_cycle, "status_words": status,
            "launch_plans": plans}


def bench_served(seconds: float, speedups, budget: int, n_streams: int = 64, rate_hz: float = 10.0,
                 pool: int = 4, realtime_seconds: float = 10.0):
    """64 streams of sizes drawn from {128^2, 256^2, 512^2} (8 particles and one new-born slot
    per cell), each receiving measurement grids as a Poisson process of `rate_hz` over `seconds`
    of simulated time, replayed at each speed in `speedups` through the serving runtime
    (admission against `budget` bytes, continuous batching); at speed 1 (real time) only the
    first `realtime_seconds` are replayed, so the run holds the GPU for about that long.  The
    speeds above the GPU's capacity show where serving saturates: the request rate stops
    following the offered load and latency grows with the queue.  Each stream cycles through
    `pool` pre-uploaded measurement grids of its own scene."""
    import numpy as np
    import torch

    from paper_1605_02406_amd import dogm, scenes
    from paper_1605_02406_amd.serve import Server

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1000)
    sizes = rng.choice([128, 256, 512], size=n_streams)
    wls = [scenes.batch_workload(int(n), seed=i) for i, n in enumerate(sizes)]
    params = [dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"],
                               seed=i, grid_id=i, **scenes.FILTER) for i, wl in enumerate(wls)]
    meas = [[dogm.Meas(torch.as_tensor(m["m_occ"], device=dev),
                       torch.as_tensor(m["m_free"], device=dev))
             for m in scenes.measurement_sequence(wl, pool)] for wl in wls]
    arrivals = []
    for i in range(n_streams):
        t = rng.exponential(1.0 / rate_hz)
        while t < seconds:
            arrivals.append((t, i))
            t += rng.exponential(1.0 / rate_hz)
    arrivals.sort()
    runs = []
    for speed in speedups:
        srv = Server(budget)
        admitted = [i for i in range(n_streams) if srv.open(i, params[i])]
        # one untimed cycle of every admitted stream
        for i in admitted:
            srv.submit(i, meas[i][0])
        srv.drain()
        srv.stats.done.clear()
        srv.stats.batches = srv.stats.batched_requests = 0
        srv.stats.batch_sizes.clear()
        count = {i: 1 for i in admitted}
        horizon = min(seconds, realtime_seconds) if speed <= 1.0 else seconds
        todo = [(t, i) for t, i in arrivals if i in count and t < horizon]
        clock = srv.clock
        # the host loop runs with Python's cyclic garbage collector paused, as a serving loop
        # would: a full collection walks the whole heap and stalls the loop for milliseconds
        gc.collect()
        gc.freeze()
        gc.disable()
        try:
            t0 = clock()
            nxt = 0
            while nxt < len(todo) or srv.pending or srv.inflight:
                now = clock()
                while nxt < len(todo) and t0 + todo[nxt][0] / speed <= now:
                    t, i = todo[nxt]
                    srv.submit(i, meas[i][count[i] % pool], t_arrival=t0 + t / speed)
                    count[i] += 1
                    nxt += 1
                srv.pump()
            wall = clock() - t0
        finally:
            gc.enable()
            gc.unfreeze()
        lat = np.array([r.latency for r in srv.stats.done]) * 1e3
        sizes_hist = {str(k): v for k, v in sorted(srv.stats.batch_sizes.items())}
        runs.append({"speedup": speed, "simulated_s": horizon, "offered_requests_per_s":
                     len(todo) / (horizon / speed), "requests": int(lat.size), "wall_s": wall,
                     "requests_per_s": lat.size / wall,
                     "particles_per_s": sum(8 * int(srv.grids[r.sid].C) for r in srv.stats.done)
                     / wall,
                     "latency_ms_p50": float(np.percentile(lat, 50)) if lat.size else None,
                     "latency_ms_p99": float(np.percentile(lat, 99)) if lat.size else None,
                     "latency_ms_max": float(lat.max()) if lat.size else None,
                     "batches": srv.stats.batches,
                     "mean_batch": srv.stats.batched_requests / max(srv.stats.batches, 1),
                     "batch_sizes": sizes_hist,
                     "streams_admitted": len(admitted),
                     "streams_rejected": srv.stats.rejected_streams,
                     "hbm_reserved_bytes": srv.admission.used,
                     "status_nonzero": sum(1 for i in admitted if srv.grids[i].status() != 0)})
        del srv
        torch.cuda.synchronize()
    return {"streams": n_streams, "sizes": {str(n): int((sizes == n).sum()) for n in (128, 256, 512)},
            "rate_hz_per_stream": rate_hz, "simulated_s": seconds, "budget_bytes": budget,
            "runs": runs}


def cpu_baseline(p, seq, budget_s):
    """The oracle (single-threaded FP64 C, as it stands) on the same workload: whole cycles from
    its own initial state until `budget_s` seconds of host time are spent, timed on this host."""
    import numpy as np

    import oracle
    op = oracle.Params(p.nx, p.ny, p.cell_size, p.dt, p.p_s, p.p_b, p.sigma_pos, p.sigma_vel,
                       p.sigma_birth_vel, p.alpha_free, p.n_pers, p.n_born, seed=p.seed)
    st = oracle.init_state(op, op.n_pers)
    m_F = np.zeros(op.C)
    n = 0
    t0 = time.perf_counter()
    while True:
        n += 1
        st, m_F, _ = oracle.cycle(op, n, st, m_F, seq[(n - 1) % len(seq)])
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n / dt, "unit": "cycles/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_cpus": os.cpu_count(),
            "sample": f"{n} cycles of the same {p.nx}x{p.ny} / {_pow2(p.n_pers)}+{_pow2(p.n_born)} "
                      f"workload from the oracle's "
                      f"own initial state ({dt:.1f} s)",
            "particles_per_s": n * op.n_pers / dt}


if __name__ == "__main__":
    main()
