"""Launch-plan autotuner: picks, for one grid shape, the plan knobs of dogm_params that make a
cycle fastest on this device, by timing every candidate plan.

The knobs change how the work is cut into launches and tiles, never a result (the sort is
stable and every prefix sum is exact), so the choice is a pure timing question:
  * sort_passes: the fewest radix passes with digits of at most 11 bits, or one more pass with
    narrower digits (smaller LDS per block, more blocks per compute unit, fewer ballots per key);
  * scan_parts: every consumer block adds up the per-tile partial sums before its own (no extra
    launch), or one small kernel scans them once (an extra launch, one read per block);
  * resample: every tile's outputs shared evenly by its threads (a binary search per output),
    or each source's draws written by the lane that owns it (cheaper per output, but a source
    with many draws is written by one lane).

    plan, report = tune(params)          # params: dogm.CParams
    params = with_plan(params, plan)

Each candidate runs on a grid of its own: `warmup` cycles, then `cycles` cycles captured as one
HIP graph each and replayed; the plan with the smallest median replay time wins.  Results are
cached per shape (grid size, particle counts, model, precision) for the life of the process.
"""
from __future__ import annotations

import ctypes as ct
import itertools

from . import dogm, scenes

MAX_DIGIT_BITS = 11
MAX_PASSES = 3

_cache: dict = {}


def fewest_passes(C: int) -> int:
    """Passes the library uses by default: keys 0..C with digits of at most 11 bits."""
    bits = max(1, C.bit_length())
    return -(-bits // MAX_DIGIT_BITS)


def candidates(params: dogm.CParams) -> list:
    C = params.nx * params.ny
    lo = fewest_passes(C)
    passes = [p for p in (lo, lo + 1) if p <= MAX_PASSES]
    return [dict(sort_passes=p, scan_parts=s, resample=r)
            for p, s, r in itertools.product(passes, (1, 2), (1, 2))]


def with_plan(params: dogm.CParams, plan: dict) -> dogm.CParams:
    q = dogm.CParams()
    ct.pointer(q)[0] = params  # copy
    q.sort_passes = plan["sort_passes"]
    q.scan_parts = plan["scan_parts"]
    q.resample = plan["resample"]
    return q


def _key(p: dogm.CParams):
    return (p.nx, p.ny, p.n_pers, p.n_born, p.model, p.precision)


def _workload(p: dogm.CParams) -> dict:
    return dict(nx=p.nx, ny=p.ny, cell=p.cell_size, n_pers=p.n_pers, n_born=p.n_born,
                scene="boxes", n_boxes=max(2, round(30 * p.nx * p.ny / 512 ** 2)), clutter=0.01,
                seed=7)


def time_plan(params: dogm.CParams, plan: dict, meas: list, warmup: int, cycles: int) -> float:
    """Median milliseconds of one replayed cycle under `plan`."""
    import numpy as np
    import torch

    g = dogm.Grid(with_plan(params, plan))
    for k in range(warmup):
        g.step(meas[k % len(meas)])
    side = torch.cuda.Stream()
    graphs = []
    for k in range(cycles):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            g.step(meas[(warmup + k) % len(meas)])
        graphs.append(gr)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in graphs]
    torch.cuda.synchronize()
    for (a, b), gr in zip(ev, graphs):
        a.record()
        gr.replay()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def tune(params: dogm.CParams, warmup: int = 4, cycles: int = 8, meas: list | None = None):
    """(best plan, {plan as text: median ms per cycle}) for the shape of `params`."""
    import torch

    key = _key(params)
    if key in _cache:
        return _cache[key]
    if meas is None:
        dev = torch.device("cuda")
        if params.model == dogm.MODEL_PHD_MIB:
            seq = scenes.measurement_sequence(_workload(params), 4, model="phd")
        else:
            seq = scenes.measurement_sequence(_workload(params), 4)
        meas = [dogm.Meas(**{k: torch.as_tensor(v, device=dev) for k, v in m.items()})
                for m in seq]
    report = {}
    best, best_ms = None, float("inf")
    for plan in candidates(params):
        ms = time_plan(params, plan, meas, warmup, cycles)
        report[f"passes={plan['sort_passes']},scan={plan['scan_parts']},"
               f"resample={plan['resample']}"] = ms
        if ms < best_ms:
            best, best_ms = plan, ms
    _cache[key] = (best, report)
    return best, report
