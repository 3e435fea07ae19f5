"""Precision study on the 1024x1024 grid at 0.1 m with 2^23 persistent and 2^20 new-born
particles (GPU script, not collected by pytest):

    python tests/precision_study.py [--cycles 4] [--out profiles/precision_c1024]

For each precision mode the grid runs cycles 1..K-1 and the K-th cycle call by call against
the oracle (tests/parity.py), recording the maximum and the 99th percentile of every output's
scaled error.  On the resampling call's own inputs it also evaluates two CDF variants on the
host next to the exact fixed-point CDF both sides use: a plain sequential FP64 sum and a
sequential FP32 sum, and counts the resampling indices each would choose differently and the
largest change of a cell's resampled particle count.  Writes <out>.json and <out>.md."""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
from paper_1605_02406_amd import dogm, scenes  # noqa: E402
from tests import parity  # noqa: E402
from tests.parity import PerCall, device_meas, host, oracle_params, u32  # noqa: E402


def cdf_variants(p, k, g):
    """Resampling indices of the exact fixed-point CDF against plain FP64 and FP32 CDFs, on the
    sorted persistent and new-born weights the resampling call receives."""
    wp = host(g.v["sw"]).astype(np.float64)
    wb = host(g.v["bw"]).astype(np.float64)
    U = oracle.resample_offset(p, k)
    idx_fix, W = oracle.resample_indices(wp, wb, U)
    nu = p.n_pers
    wj = np.concatenate([wp, wb])
    skey = np.concatenate([u32(g.v["skey"]), u32(g.v["bkey"])]).astype(np.int64)
    out = {}
    for name, dt in (("fp64_plain_cdf", np.float64), ("fp32_cdf", np.float32)):
        F = np.cumsum(wj.astype(dt), dtype=dt)
        u = ((np.arange(nu, dtype=np.float64) + U).astype(dt) * (F[-1] / dt(nu))).astype(dt)
        idx = np.minimum(np.searchsorted(F, u, side="right"), len(wj) - 1)
        diff = int((idx != idx_fix).sum())
        cnt_fix = np.bincount(skey[idx_fix], minlength=p.C + 1)
        cnt = np.bincount(skey[idx], minlength=p.C + 1)
        out[name] = {"indices_differing": diff, "fraction": diff / nu,
                     "max_cell_count_change": int(np.abs(cnt - cnt_fix)[:p.C].max()),
                     "cells_changed": int((cnt != cnt_fix)[:p.C].sum())}
    out["W"] = W * 2.0 ** -40
    return out


def study(mode, cycles):
    wl = scenes.WORKLOADS["c1024"]
    prm = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"],
                           precision=mode, **scenes.FILTER)
    g = dogm.Grid(prm)
    pc = PerCall(g)
    seq = scenes.measurement_sequence(wl, cycles)
    for k, m in enumerate(seq[:-1], start=1):
        g.step(device_meas(m))
    k = cycles
    parity.P99.clear()
    pc.predict()
    pc.assign()
    pc.update(device_meas(seq[-1]))
    pc.moments()
    variants = cdf_variants(oracle_params(prm), k, g)
    pc.resample()
    torch.cuda.synchronize()
    rows = {}
    for key, mx in pc.stats.items():
        if isinstance(mx, float):
            short = key.split(".", 1)[1]
            rows[key] = {"max": mx, "p99": parity.P99.get(
                {"predict": f"predict {short}", "update": f"update {short}",
                 "born": f"born {short}", "moments": short}[key.split(".")[0]], None)}
    return {"mode": "FP64" if mode else "FP32", "cycle": k, "errors": rows,
            "resample_cdf_variants": variants, "status": g.status()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cycles", type=int, default=4)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "precision_c1024"))
    a = ap.parse_args()
    res = [study(m, a.cycles) for m in (dogm.PRECISION_FP32, dogm.PRECISION_FP64)]
    rec = {"workload": "1024x1024 grid at 0.1 m, 2^23 persistent + 2^18 new-born particles",
           "command": "python tests/precision_study.py --cycles %d" % a.cycles, "modes": res}
    rec["workload"] = rec["workload"].replace("2^18", "2^20")
    with open(a.out + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [f"# Precision study, {rec['workload']}", "", "Command (MI355X, one GPU):", "",
             "    " + rec["command"], "",
             f"Errors of every call of cycle {a.cycles} against the oracle on the call's own inputs "
             "(scaled as in tests/parity.py: positions and velocities by max(|ref|, 1), masses by "
             "max(|ref|, 1e-4), weights by |ref|, variances by the raw second moment).", "",
             "| output | FP32 max | FP32 p99 | FP64 max | FP64 p99 |", "|---|---|---|---|---|"]
    for key in res[0]["errors"]:
        e32, e64 = res[0]["errors"][key], res[1]["errors"].get(key, {})
        fmt = lambda v: "—" if v is None else f"{v:.2e}"  # noqa: E731
        lines.append(f"| {key} | {fmt(e32['max'])} | {fmt(e32['p99'])} | {fmt(e64.get('max'))} | "
                     f"{fmt(e64.get('p99'))} |")
    lines += ["", "Resampling indices against the exact fixed-point CDF (on each mode's own "
              "weights of the same call):", "",
              "| mode | CDF | indices differing | fraction | cells whose count changes | "
              "largest count change |", "|---|---|---|---|---|---|"]
    for r in res:
        for name, v in r["resample_cdf_variants"].items():
            if name == "W":
                continue
            lines.append(f"| {r['mode']} | {name} | {v['indices_differing']} | {v['fraction']:.2e} | "
                         f"{v['cells_changed']} | {v['max_cell_count_change']} |")
    with open(a.out + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
