"""Filter-quality evaluation on a synthetic scene with known truth (Sec. VIII).

The paper evaluates the filter on recorded laser data: the mean velocity of the cells of a moving
object (eq. (mean_cluster)), the spread of that estimate as a Gaussian mixture over the object's
cells (eq. (gaussian_mixture_x)), the normalised estimation error squared (eq. (NEES_x)) against
the 95 % level, and the separation of moving from stationary cells by the Mahalanobis distance of
the cell velocity from zero (eq. (mahadist)) as a ROC curve; each under p_B in {0.005, 0.02, 0.1}.
Here the same quantities are computed from the GPU filter's moments on a synthetic scene whose
truth is known: parked cars along two lanes, cars and a smaller object driving along x through
the lanes and turning back at the grid border (a manoeuvre the constant-velocity model does not
describe), and static clutter.

Readings where the paper leaves a choice (each also in the design notes):
  * S, the cells of an object: the cells whose centre lies in the object's box and whose moments
    are defined (they hold particles with weight);
  * the classified cells are the truth-occupied cells with a detection in that cycle: the paper's
    ROC is over labelled measurement points (returns on static and on moving objects); a cell
    holding fewer than three particles (whose two-dimensional covariance is singular) or without
    defined moments counts as a static detection (m = 0); P is regularised by 1e-6 (m/s)^2 I
    before the inversion.  The ROC under other readings (every truth-occupied cell with at
    least three particles, every one with moments, only cells the map holds as occupied) is
    reported beside it: the truth-occupied cells the sensor does not see (the far sides and
    interiors of objects) hold a few particles of little mass (rho_p about 0.01 against 0.09 for
    static cells as a whole, at p_B = 0.02) whose mean velocity is that of a few new-born
    particles, and they supply nearly all static cells with large m;
  * the x-axis is the driving direction, so the x-components are evaluated as in the paper.

    python -m paper_1605_02406_amd.evaluate [--cycles N] [--p-b 0.005,0.02,0.1] [--model ds,phd]
    python -m paper_1605_02406_amd.evaluate --approach     # NEES per phase of an approach
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import scenes

CHI2_1_95 = 3.841458820694124  # 95 % quantile of chi^2 with one degree of freedom
PRIMARY_READING = "detected"


# -- metrics (plain functions of the per-cell moments) ----------------------------------------

def cluster_mean(mean_x: np.ndarray) -> float:
    """eq. (mean_cluster): unweighted mean of the cell means over the object's cells."""
    return float(np.mean(mean_x))


def cluster_variance(mean_x: np.ndarray, var_x: np.ndarray) -> float:
    """eq. (gaussian_mixture_x): variance of the equal-weight Gaussian mixture of the cells."""
    m = cluster_mean(mean_x)
    return float(np.mean(var_x + mean_x * mean_x) - m * m)


def nees(estimate: float, variance: float, truth: float) -> float:
    """eq. (NEES_x): squared error of the estimate normalised by its variance."""
    return (estimate - truth) ** 2 / variance


def mahalanobis(mx, my, vxx, vyy, vxy, reg: float = 1e-6) -> np.ndarray:
    """eq. (mahadist): m = v P^-1 v^T for each cell, P = [[vxx, vxy], [vxy, vyy]] + reg I."""
    a = np.asarray(vxx, np.float64) + reg
    d = np.asarray(vyy, np.float64) + reg
    b = np.asarray(vxy, np.float64)
    mx = np.asarray(mx, np.float64)
    my = np.asarray(my, np.float64)
    det = a * d - b * b
    with np.errstate(divide="ignore", invalid="ignore"):
        m = (d * mx * mx - 2.0 * b * mx * my + a * my * my) / det
    return np.where(det > 0, m, np.inf)


def roc(score: np.ndarray, dynamic: np.ndarray):
    """ROC of 'dynamic if score >= tau' over every threshold: (false positive rates, true
    positive rates), both starting at (0, 0) and ending at (1, 1)."""
    score = np.asarray(score, np.float64)
    dynamic = np.asarray(dynamic, bool)
    n_pos, n_neg = int(dynamic.sum()), int((~dynamic).sum())
    if n_pos == 0 or n_neg == 0:
        raise ValueError("the ROC needs dynamic and static cells")
    order = np.argsort(-score, kind="stable")
    s, d = score[order], dynamic[order]
    tp = np.cumsum(d)
    fp = np.cumsum(~d)
    last = np.r_[s[1:] != s[:-1], True]  # one point per distinct threshold
    tpr = np.r_[0.0, tp[last] / n_pos]
    fpr = np.r_[0.0, fp[last] / n_neg]
    return fpr, tpr


def auc(fpr: np.ndarray, tpr: np.ndarray) -> float:
    return float(np.sum((fpr[1:] - fpr[:-1]) * (tpr[1:] + tpr[:-1]) / 2.0))


def tpr_at_fpr(fpr: np.ndarray, tpr: np.ndarray, level: float) -> float:
    """Highest true positive rate of a threshold whose false positive rate is <= level."""
    ok = fpr <= level
    return float(tpr[ok].max()) if ok.any() else 0.0


# -- the evaluation scene ---------------------------------------------------------------------

def lanes_scene(nx: int = 320, ny: int = 160, cell: float = 0.2, seed: int = 0) -> scenes.Scene:
    """64 m x 32 m at 0.2 m, sensor in the centre: parked cars (4.5 m x 1.8 m, static) along
    both sides of two lanes, two cars (8 m/s and 5 m/s) and a smaller object (1.0 m x 0.8 m,
    3 m/s) driving along x, and 0.3 % static clutter cells."""
    W, H = nx * cell, ny * cell
    boxes = []
    for y in (0.2 * H, 0.8 * H):
        for x in np.arange(0.1, 1.0, 0.125) * W:
            if abs(x - W / 2) > 6.0:
                boxes.append(scenes.Box(float(x), float(y), 4.5, 1.8, 0.0, 0.0))
    moving = [scenes.Box(0.2 * W, 0.35 * H, 4.5, 1.8, 8.0, 0.0),
              scenes.Box(0.75 * W, 0.65 * H, 4.5, 1.8, -5.0, 0.0),
              scenes.Box(0.6 * W, 0.42 * H, 1.0, 0.8, 3.0, 0.0)]
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1605, 8]))
    clutter = rng.random((ny, nx)) < 0.003
    cy0, cx0 = ny // 2, nx // 2
    clutter[cy0 - 3:cy0 + 3, cx0 - 3:cx0 + 3] = False
    return scenes.Scene(nx, ny, cell, boxes + moving, clutter=clutter, seed=seed)


def _box_cells(sc: scenes.Scene, b: scenes.Box) -> np.ndarray:
    xc = (np.arange(sc.nx) + 0.5) * sc.cell
    yc = (np.arange(sc.ny) + 0.5) * sc.cell
    ix = (xc >= b.cx - b.w / 2) & (xc <= b.cx + b.w / 2)
    iy = (yc >= b.cy - b.h / 2) & (yc <= b.cy + b.h / 2)
    return (iy[:, None] & ix[None, :]).reshape(-1)


# -- the run ----------------------------------------------------------------------------------

def evaluate(p_b: float, cycles: int = 80, warmup: int = 20, n_pers: int = 1 << 19,
             n_born: int = 1 << 16, seed: int = 0, model: str = "ds") -> dict:
    """Runs the GPU filter (the Dempster-Shafer model, "ds", or the particle PHD/MIB model of
    Sec. V, "phd") on the lanes scene for `cycles` cycles and returns the metrics over the
    cycles after `warmup`."""
    import torch

    from . import dogm

    sc = lanes_scene(seed=seed)
    filt = dict(scenes.FILTER)
    filt["p_b"] = p_b
    p = dogm.make_params(sc.nx, sc.ny, sc.cell, n_pers, n_born, seed=seed,
                         model=dogm.MODEL_PHD_MIB if model == "phd" else dogm.MODEL_DS, **filt)
    g = dogm.Grid(p)
    moving = [b for b in sc.boxes if b.vx != 0.0 or b.vy != 0.0]
    rows, scores, labels, counts, pigns, dets = [], [], [], [], [], []
    lost, born_total = 0.0, 0.0  # new-born mass on cells whose share of the slots rounds to none
    for k in range(1, cycles + 1):
        sc.advance()
        occ = sc.truth().reshape(-1)
        rng = np.random.default_rng(np.random.SeedSequence([seed, k, 99]))
        if model == "phd":
            obs = scenes.detection_grid(occ.reshape(sc.ny, sc.nx), rng)
        else:
            m_occ, m_free = scenes.measurement_grid(occ.reshape(sc.ny, sc.nx), rng)
            obs = dict(m_occ=m_occ, m_free=m_free)
        meas = dogm.Meas(**{k: torch.as_tensor(v, device="cuda") for k, v in obs.items()})
        g.step(meas)
        if k <= warmup:
            continue
        rho_b = g.v["rho_b"].cpu().numpy().astype(np.float64)
        off = g.v["born_off"].cpu().numpy().astype(np.int64)
        lost += float(rho_b[(rho_b > 0) & (off[1:] == off[:-1])].sum())
        born_total += float(rho_b.sum())
        mx = g.v["mean_x"].cpu().numpy()
        my = g.v["mean_y"].cpu().numpy()
        vxx = g.v["var_x"].cpu().numpy()
        vyy = g.v["var_y"].cpu().numpy()
        vxy = g.v["cov_xy"].cpu().numpy()
        defined = g.v["mom_flag"].cpu().numpy() != 0
        count = (g.v["cell_end"].cpu().numpy().astype(np.int64) -
                 g.v["cell_start"].cpu().numpy().astype(np.int64))
        pign = g.v["pign"].cpu().numpy()
        dyn = np.zeros(occ.shape, bool)
        for i, b in enumerate(moving):
            cells = _box_cells(sc, b)
            dyn |= cells
            S = cells & defined
            if not S.any():
                continue
            est = cluster_mean(mx[S])
            var = cluster_variance(mx[S].astype(np.float64), vxx[S].astype(np.float64))
            rows.append(dict(cycle=k, obj=i, truth=b.vx, est=est, var=var,
                             nees=nees(est, var, b.vx) if var > 0 else math.inf))
        m = np.where(defined, mahalanobis(mx, my, vxx, vyy, vxy), 0.0)
        scores.append(m[occ])
        labels.append(dyn[occ])
        counts.append(count[occ])
        pigns.append(pign[occ])
        dets.append(np.asarray(obs["m_occ"] if model != "phd" else obs["det"])[occ] > 0)
    # births in every cell (Sec. V) leave cells without a slot: not an error there
    allowed = dogm.ST_NOCARRIER if model == "phd" else 0
    if g.status() & ~allowed:
        raise RuntimeError(f"filter status word {g.status():#x}")
    score, label = np.concatenate(scores), np.concatenate(labels)
    count, pign, det = np.concatenate(counts), np.concatenate(pigns), np.concatenate(dets)
    # a velocity distribution in two dimensions needs at least three particles; the map holds a
    # cell as occupied when its pignistic occupancy exceeds one half
    readings = {"detected": det & (count >= 3),
                "all_occupied": np.ones(score.shape, bool), "three_particles": count >= 3,
                "map_occupied": pign > 0.5, "three_particles_map_occupied": (count >= 3) & (pign > 0.5)}
    roc_out = {}
    for name, keep in readings.items():
        if name == "detected":  # the classified set is the detected cells themselves
            f, t = roc(np.where(count >= 3, score, 0.0)[det], label[det])
        else:  # cells outside the reading count as static detections
            f, t = roc(np.where(keep, score, 0.0), label)
        roc_out[name] = {"auc": auc(f, t), "tpr_at_fpr_1pct": tpr_at_fpr(f, t, 0.01)}
    fpr, tpr = roc(np.where(count >= 3, score, 0.0)[det], label[det])
    err = np.array([r["est"] - r["truth"] for r in rows])
    toward = np.array([(r["est"] - r["truth"]) * math.copysign(1.0, r["truth"]) for r in rows])
    nv = np.array([r["nees"] for r in rows])
    sd = np.sqrt(np.array([r["var"] for r in rows]))
    return {"model": model, "p_b": p_b, "cycles": cycles, "warmup": warmup, "samples": len(rows),
            "velocity_mae_mps": float(np.mean(np.abs(err))),
            "velocity_bias_along_motion_mps": float(np.mean(toward)),
            "velocity_sd_mps": float(np.mean(sd)),
            "nees_median": float(np.median(nv)),
            "nees_frac_above_95pct": float(np.mean(nv > CHI2_1_95)),
            "roc_auc": auc(fpr, tpr),
            "tpr_at_fpr_1pct": tpr_at_fpr(fpr, tpr, 0.01),
            "roc_readings": roc_out,
            "cells_dynamic": int(label[det].sum()), "cells_static": int((~label[det]).sum()),
            "new_born_mass_without_slot_frac": lost / born_total if born_total > 0 else 0.0}


# -- an approaching object with acceleration and deceleration (Sec. VIII.B) -------------------

# The paper's scenario: a small object approaches the sensor from far away, accelerates slowly,
# drives at an almost constant speed, then decelerates strongly.  Phases of the synthetic
# profile (cycles of T = 0.1 s, the object at rest before and after):
APPROACH_PHASES = (("rest", 20, 0.0), ("accelerate", 40, 0.1), ("cruise", 30, 0.0),
                   ("decelerate", 10, -0.4), ("stopped", 20, 0.0))  # (name, cycles, dv per cycle)


def approach_profile():
    """(phase name, truth velocity in m/s) of every cycle: 1 m/s^2 up to 4 m/s, then 4 m/s^2
    down to rest."""
    out, v = [], 0.0
    for name, n, dv in APPROACH_PHASES:
        for _ in range(n):
            v = max(0.0, round(v + dv, 9))
            out.append((name, v))
    return out


def evaluate_approach(p_b: float, n_pers: int = 1 << 19, n_born: int = 1 << 16, seed: int = 0,
                      model: str = "ds", settle: int = 5, noise: dict | None = None) -> dict:
    """NEES and velocity error of the approaching object per phase of its profile.  The object
    (1.0 m x 0.8 m) drives along x towards the sensor on the lanes scene; rows of a phase skip
    its first `settle` cycles only for the rest phase (the filter's start-up).  `noise`
    overrides filter parameters (e.g. the process noise of the paper's Table I)."""
    import torch

    from . import dogm

    sc = lanes_scene(seed=seed)
    W, H = sc.size
    obj = scenes.Box(4.0, 0.5 * H + 1.6, 1.0, 0.8, 0.0, 0.0)
    sc.boxes.append(obj)
    filt = dict(scenes.FILTER)
    filt.update(noise or {})
    filt["p_b"] = p_b
    p = dogm.make_params(sc.nx, sc.ny, sc.cell, n_pers, n_born, seed=seed,
                         model=dogm.MODEL_PHD_MIB if model == "phd" else dogm.MODEL_DS, **filt)
    g = dogm.Grid(p)
    rows = []
    for k, (phase, v) in enumerate(approach_profile(), start=1):
        obj.vx = v
        sc.advance()
        occ = sc.truth().reshape(-1)
        rng = np.random.default_rng(np.random.SeedSequence([seed, k, 98]))
        if model == "phd":
            obs = scenes.detection_grid(occ.reshape(sc.ny, sc.nx), rng)
        else:
            m_occ, m_free = scenes.measurement_grid(occ.reshape(sc.ny, sc.nx), rng)
            obs = dict(m_occ=m_occ, m_free=m_free)
        g.step(dogm.Meas(**{kk: torch.as_tensor(vv, device="cuda") for kk, vv in obs.items()}))
        if phase == "rest" and k <= settle:
            continue
        defined = g.v["mom_flag"].cpu().numpy() != 0
        detected = np.asarray(obs["det"] if model == "phd" else obs["m_occ"]) > 0
        mx_all = g.v["mean_x"].cpu().numpy().astype(np.float64)
        vxx_all = g.v["var_x"].cpu().numpy().astype(np.float64)
        # two readings of S: every cell of the box with moments, and only those with a detection
        # in this cycle (the object's returns)
        for reading, S in (("box", _box_cells(sc, obj) & defined),
                           ("detected", _box_cells(sc, obj) & defined & detected)):
            if not S.any():
                continue
            est, var = cluster_mean(mx_all[S]), cluster_variance(mx_all[S], vxx_all[S])
            rows.append(dict(reading=reading, phase=phase, truth=v, est=est, var=var,
                             nees=nees(est, var, v) if var > 0 else math.inf))
    out = {"model": model, "p_b": p_b, "noise": {k: filt[k] for k in ("sigma_pos", "sigma_vel")},
           "phases": {}, "phases_detected_cells": {}}
    for reading, key in (("box", "phases"), ("detected", "phases_detected_cells")):
        for name, _, _ in APPROACH_PHASES:
            r = [x for x in rows if x["phase"] == name and x["reading"] == reading]
            if not r:
                continue
            nv = np.array([x["nees"] for x in r])
            err = np.array([x["est"] - x["truth"] for x in r])
            out[key][name] = {"samples": len(r), "nees_mean": float(np.mean(nv)),
                              "nees_frac_above_95pct": float(np.mean(nv > CHI2_1_95)),
                              "velocity_error_mean_mps": float(np.mean(err)),
                              "velocity_sd_mps": float(np.mean([math.sqrt(x["var"]) for x in r]))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cycles", type=int, default=80)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--p-b", default="0.005,0.02,0.1")
    ap.add_argument("--model", default="ds,phd", help="ds, phd or both")
    ap.add_argument("--approach", action="store_true",
                    help="the approaching object's phases instead of the lanes metrics")
    ap.add_argument("--sigma-pos", type=float, default=None, help="process noise, position (m)")
    ap.add_argument("--sigma-vel", type=float, default=None, help="process noise, velocity (m/s)")
    args = ap.parse_args()
    for model in [m for m in args.model.split(",") if m]:
        for pb in [float(x) for x in args.p_b.split(",") if x]:
            if args.approach:
                noise = {k: v for k, v in (("sigma_pos", args.sigma_pos),
                                           ("sigma_vel", args.sigma_vel)) if v is not None}
                print(json.dumps(evaluate_approach(pb, model=model, noise=noise)), flush=True)
            else:
                print(json.dumps(evaluate(pb, args.cycles, args.warmup, model=model)), flush=True)


if __name__ == "__main__":
    main()
