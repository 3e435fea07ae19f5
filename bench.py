#!/usr/bin/env python3
"""Throughput of the DS-PHD/MIB particle recursion on one MI355X.

A step is one full filter cycle (predict, assign, update, moments, resample) of the 512x512 grid
at 0.2 m with 2^21 persistent and 2^18 new-born particles over a synthetic ray-cast scene
(30 moving boxes, 1 % static clutter).  Measurement grids are generated and uploaded before the
timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "filter cycles/s and particles/s at 512²/2M; p50/p99 cycle latency multi-stream"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes (each array read / written once per step that needs it, the sort as one
# ideal pass, random numbers in registers): per persistent particle, per new-born slot, per cell.
B_PER_PARTICLE = 156
B_PER_BORN = 28
B_PER_CELL = 92
# predict reads x, y, vx, vy, w and writes them plus the key
PREDICT_BYTES_PER_PARTICLE = 20 + 24


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c512")
    ap.add_argument("--cpu-cycles", type=int, default=20,
                    help="oracle cycles timed on the host for the CPU baseline (0: skip)")
    ap.add_argument("--events", action="store_true", default=True)
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU: the filter of one grid does not span GPUs here "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1605_02406_amd import dogm, scenes

    wl = scenes.WORKLOADS[args.workload]
    p = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"],
                         seed=wl.get("seed", 0), **scenes.FILTER)
    C = wl["nx"] * wl["ny"]
    n_cycles = args.warmup + args.steps
    t_gen = time.perf_counter()
    seq = scenes.measurement_sequence(wl, n_cycles)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    meas = [dogm.Meas(torch.as_tensor(m["m_occ"], device=dev),
                      torch.as_tensor(m["m_free"], device=dev)) for m in seq]
    g = dogm.Grid(p)
    torch.cuda.synchronize()

    for k in range(args.warmup):
        g.step(meas[k])
    torch.cuda.synchronize()

    # timed region: every call of every step, with HIP events between the calls on the
    # grid's stream (the current stream)
    names = ["predict", "assign", "update", "moments", "resample"]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
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
    wall = time.perf_counter() - t0
    status = g.status()

    per_call = {n: float(np.mean([ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(args.steps)]))
                for i, n in enumerate(names)}
    cycle_ms = [ev[s][0].elapsed_time(ev[s][5]) for s in range(args.steps)]
    ms_per_step = wall * 1e3 / args.steps
    cycles_per_s = args.steps / wall
    nu, nb = wl["n_pers"], wl["n_born"]
    b_alg = B_PER_PARTICLE * nu + B_PER_BORN * nb + B_PER_CELL * C

    pred_ms = per_call["predict"]
    pred_gbs = PREDICT_BYTES_PER_PARTICLE * nu / (pred_ms * 1e-3) / 1e9

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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 grid at 0.2 m, 2^21 persistent + 2^18 new-born "
                               "particles, ray-cast scene of 30 moving boxes + 1% clutter",
                   "nx": wl["nx"], "ny": wl["ny"], "cell_m": wl["cell"], "n_pers": nu,
                   "n_born": nb},
        "particles_per_s": cycles_per_s * nu,
        "all_particles_per_s": cycles_per_s * (nu + nb),
        "cycle_ms_p50": float(np.percentile(cycle_ms, 50)),
        "cycle_ms_p99": float(np.percentile(cycle_ms, 99)),
        "per_call_ms": per_call,
        "cycle_roofline": {"bound": "hbm", "algorithmic_bytes": b_alg,
                           "achieved": b_alg / (ms_per_step * 1e-3) / 1e9,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": b_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {"kernel": "k_predict", "bound": "hbm", "achieved": pred_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": pred_gbs / HBM_PEAK_GBS,
                     "traffic": None},
        "status_word": status,
        "meas_generation_s": t_gen,
    }

    if args.cpu_cycles > 0:
        out["cpu_baseline"] = cpu_baseline(wl, p, seq, args.cpu_cycles)
    print(json.dumps(out), flush=True)


def cpu_baseline(wl, p, seq, n):
    """The oracle (single-threaded FP64 C, as it stands) on the same workload: n cycles from its
    own initial state, timed on this host."""
    import numpy as np

    import oracle
    op = oracle.Params(p.nx, p.ny, p.cell_size, p.dt, p.p_s, p.p_b, p.sigma_pos, p.sigma_vel,
                       p.sigma_birth_vel, p.alpha_free, p.n_pers, p.n_born, seed=p.seed)
    st = oracle.init_state(op, op.n_pers)
    m_F = np.zeros(op.C)
    t0 = time.perf_counter()
    for k in range(1, n + 1):
        st, m_F, _ = oracle.cycle(op, k, st, m_F, seq[(k - 1) % len(seq)])
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} cycles of the same 512x512 / 2^21+2^18 workload from the oracle's "
                      f"own initial state ({dt:.1f} s)",
            "particles_per_s": n * op.n_pers / dt}


if __name__ == "__main__":
    main()
