"""Seeded synthetic inputs: moving-box scenes and ray-cast Dempster-Shafer measurement grids.

These stand in for the recorded laser/radar sequences of the paper's evaluation, which are
not available.  The module holds none of the filter's arithmetic: it only builds the inputs
(scene truth, measurement grids, arbitrary particle states for edge-case tests) that the GPU
library, its tests and the benchmark consume.

Measurement model (a reading; the paper's measurement-grid reference is not at hand):
  * the sensor sits at the grid centre; a 2D ray is cast to the centre of every perimeter
    cell with the Amanatides-Woo grid traversal; cells up to and including the first
    truth-occupied cell are observed, cells behind it are not;
  * each observed cell independently reports a detection with probability p_D if occupied
    and p_cl (clutter) if free, matching the paper's per-cell observation process;
  * the evidence masses are chosen so that the pignistic transform of the measurement grid
    equals the Bayesian occupancy with a uniform prior:
      detection    : P = p_D/(p_D+p_cl)          -> (m_O, m_F) = (2P-1, 0)
      no detection : P = (1-p_D)/(2-p_D-p_cl)    -> (m_O, m_F) = (0, 1-2P)
      unobserved   : (0, 0)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Filter parameters shared by every workload: time step, persistence, birth, process noise
# (per step), new-born velocity SD (Table I), free-mass discount.
FILTER = dict(dt=0.1, p_s=0.99, p_b=0.02, sigma_pos=0.1, sigma_vel=0.5, sigma_birth_vel=4.0,
              alpha_free=0.9)
SENSOR = dict(p_d=0.9, p_cl=0.01)

# Workloads.  "small": 64x64 / 32768+8192; "c512": 512x512 / 2^21+2^18; "c1024": 1024x1024 at
# 0.1 m / 2^23+2^20.
WORKLOADS = {
    "small": dict(nx=64, ny=64, cell=0.2, n_pers=32768, n_born=8192, cycles=20,
                  scene="walls", seed=0),
    "c512": dict(nx=512, ny=512, cell=0.2, n_pers=2 ** 21, n_born=2 ** 18, cycles=100,
                 scene="boxes", n_boxes=30, clutter=0.01, seed=0),
    "c1024": dict(nx=1024, ny=1024, cell=0.1, n_pers=2 ** 23, n_born=2 ** 20, cycles=50,
                  scene="boxes", n_boxes=80, clutter=0.01, seed=0),
}

# Mixed batch of 16 grids: 4x128^2, 4x256^2, 3x384^2, 3x512^2, 2x768^2, ~8 particles per cell.
BATCH_SIZES = [128] * 4 + [256] * 4 + [384] * 3 + [512] * 3 + [768] * 2


def batch_workload(n: int, seed: int) -> dict:
    return dict(nx=n, ny=n, cell=0.2, n_pers=8 * n * n, n_born=n * n, cycles=100,
                scene="boxes", n_boxes=max(2, round(30 * (n * n) / 512 ** 2)), clutter=0.01,
                seed=seed)


def mass_levels(p_d: float = SENSOR["p_d"], p_cl: float = SENSOR["p_cl"]):
    """(m_O of a detection, m_F of an observed cell without detection)."""
    P_hit = p_d / (p_d + p_cl)
    P_miss = (1.0 - p_d) / ((1.0 - p_d) + (1.0 - p_cl))
    return 2.0 * P_hit - 1.0, 1.0 - 2.0 * P_miss


@dataclass
class Box:
    cx: float
    cy: float
    w: float  # extent along x
    h: float  # extent along y
    vx: float
    vy: float


@dataclass
class Scene:
    nx: int
    ny: int
    cell: float
    boxes: list
    walls: list = field(default_factory=list)  # static rectangles (x0, y0, x1, y1)
    clutter: np.ndarray | None = None  # static occupied cells, bool [ny, nx]
    dt: float = FILTER["dt"]
    seed: int = 0
    # half-width of a square around the sensor (grid centre) that boxes never enter: they
    # reflect off it as off the border, so no box can cover the sensor and blind every ray
    keepout: float = 0.0

    @property
    def size(self):
        return self.nx * self.cell, self.ny * self.cell

    def _reflect_off_sensor(self, b: Box):
        """Push a box that overlaps the keep-out square back out along the axis it entered the
        least, mirrored, with that velocity component pointing away from the sensor."""
        if self.keepout <= 0.0:
            return
        W, H = self.size
        sx, sy = W / 2, H / 2
        px = b.w / 2 + self.keepout - abs(b.cx - sx)  # overlap along x
        py = b.h / 2 + self.keepout - abs(b.cy - sy)
        if px <= 0.0 or py <= 0.0:
            return
        if px <= py:
            side = 1.0 if b.cx >= sx else -1.0
            b.cx += side * 2.0 * px
            b.vx = side * abs(b.vx)
        else:
            side = 1.0 if b.cy >= sy else -1.0
            b.cy += side * 2.0 * py
            b.vy = side * abs(b.vy)

    def advance(self):
        """Move every box by one time step, reflecting off the keep-out square around the
        sensor and at the grid border."""
        W, H = self.size
        for b in self.boxes:
            b.cx += b.vx * self.dt
            b.cy += b.vy * self.dt
            self._reflect_off_sensor(b)
            if b.cx - b.w / 2 < 0:
                b.cx, b.vx = b.w / 2 + (b.w / 2 - b.cx), abs(b.vx)
            if b.cx + b.w / 2 > W:
                b.cx, b.vx = W - b.w / 2 - (b.cx + b.w / 2 - W), -abs(b.vx)
            if b.cy - b.h / 2 < 0:
                b.cy, b.vy = b.h / 2 + (b.h / 2 - b.cy), abs(b.vy)
            if b.cy + b.h / 2 > H:
                b.cy, b.vy = H - b.h / 2 - (b.cy + b.h / 2 - H), -abs(b.vy)

    def rects(self) -> np.ndarray:
        """The walls and boxes as float64 rectangles [n, 4] (x0, y0, x1, y1)."""
        r = list(self.walls) + [(b.cx - b.w / 2, b.cy - b.h / 2, b.cx + b.w / 2, b.cy + b.h / 2)
                                for b in self.boxes]
        return np.array(r, np.float64).reshape(-1, 4)

    def static_mask(self) -> np.ndarray:
        """Static occupied cells other than walls (bool [ny, nx])."""
        return (np.zeros((self.ny, self.nx), bool) if self.clutter is None
                else self.clutter.copy())

    def truth(self) -> np.ndarray:
        """Occupied cells (bool [ny, nx]): cell centre inside a box, a wall or clutter."""
        xc = (np.arange(self.nx) + 0.5) * self.cell
        yc = (np.arange(self.ny) + 0.5) * self.cell
        occ = np.zeros((self.ny, self.nx), bool) if self.clutter is None else self.clutter.copy()
        for (x0, y0, x1, y1) in self.walls + [(b.cx - b.w / 2, b.cy - b.h / 2, b.cx + b.w / 2,
                                               b.cy + b.h / 2) for b in self.boxes]:
            ix = (xc >= x0) & (xc <= x1)
            iy = (yc >= y0) & (yc <= y1)
            occ |= iy[:, None] & ix[None, :]
        return occ

    def velocity_truth(self) -> tuple:
        """Per-cell true velocity (0 for static cells), float [ny, nx] each."""
        xc = (np.arange(self.nx) + 0.5) * self.cell
        yc = (np.arange(self.ny) + 0.5) * self.cell
        vx = np.zeros((self.ny, self.nx))
        vy = np.zeros((self.ny, self.nx))
        for b in self.boxes:
            ix = (xc >= b.cx - b.w / 2) & (xc <= b.cx + b.w / 2)
            iy = (yc >= b.cy - b.h / 2) & (yc <= b.cy + b.h / 2)
            m = iy[:, None] & ix[None, :]
            vx[m], vy[m] = b.vx, b.vy
        return vx, vy


def _place_boxes(rng, nx, ny, cell, sizes, vels, keepout=3.0, tries=2000):
    W, H = nx * cell, ny * cell
    sx, sy = W / 2, H / 2
    boxes = []
    for (w, h), (vx, vy) in zip(sizes, vels):
        w, h = min(w, 0.5 * W), min(h, 0.5 * H)  # keep every box placeable on small grids
        for _ in range(tries):
            cx = rng.uniform(w / 2, W - w / 2)
            cy = rng.uniform(h / 2, H - h / 2)
            if (abs(cx - sx) < w / 2 + keepout) and (abs(cy - sy) < h / 2 + keepout):
                continue
            if any(abs(cx - b.cx) < (w + b.w) / 2 and abs(cy - b.cy) < (h + b.h) / 2
                   for b in boxes):
                continue
            boxes.append(Box(cx, cy, w, h, vx, vy))
            break
    return boxes


def make_scene(wl: dict, seed: int | None = None) -> Scene:
    seed = wl.get("seed", 0) if seed is None else seed
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1605, 2406]))
    nx, ny, cell = wl["nx"], wl["ny"], wl["cell"]
    W, H = nx * cell, ny * cell
    if wl["scene"] == "walls":
        # 3 boxes 1.8 x 4.5 m (long side along x), velocity components U[-10, 10] m/s, and
        # 2 static walls 0.4 m thick over the middle 60 % of the width at 20 % / 80 % height.
        sizes = [(4.5, 1.8)] * 3
        vels = [tuple(rng.uniform(-10, 10, 2)) for _ in range(3)]
        boxes = _place_boxes(rng, nx, ny, cell, sizes, vels, keepout=1.0)
        walls = [(0.2 * W, f * H - 0.2, 0.8 * W, f * H + 0.2) for f in (0.2, 0.8)]
        return Scene(nx, ny, cell, boxes, walls=walls, seed=seed, keepout=1.0)
    # boxes with sides U[0.5, 5] m, speed U[0, 20] m/s, heading U[0, 2 pi), plus static
    # clutter cells.
    nb = wl["n_boxes"]
    sizes = [tuple(rng.uniform(0.5, 5.0, 2)) for _ in range(nb)]
    vels = []
    for _ in range(nb):
        s, th = rng.uniform(0, 20), rng.uniform(0, 2 * math.pi)
        vels.append((s * math.cos(th), s * math.sin(th)))
    boxes = _place_boxes(rng, nx, ny, cell, sizes, vels)
    clutter = rng.random((ny, nx)) < wl.get("clutter", 0.0)
    cy0, cx0 = ny // 2, nx // 2
    clutter[max(cy0 - 2, 0):cy0 + 2, max(cx0 - 2, 0):cx0 + 2] = False
    return Scene(nx, ny, cell, boxes, clutter=clutter, seed=seed, keepout=3.0)


def raycast_observed(occ: np.ndarray) -> np.ndarray:
    """Cells seen from the grid centre (bool [ny, nx]): Amanatides-Woo traversal of one ray
    per perimeter cell centre, stopping at (and including) the first occupied cell.  The i-th
    boundary crossing along an axis is at t_i = t_0 + i d (one rounded product and one rounded
    sum in FP64; t_0 itself for i = 0), and each step crosses the nearer boundary, an x boundary
    only when its crossing is strictly smaller."""
    ny, nx = occ.shape
    sx, sy = nx / 2.0, ny / 2.0  # sensor position in cell units
    per = ([(i, 0) for i in range(nx)] + [(i, ny - 1) for i in range(nx)] +
           [(0, j) for j in range(1, ny - 1)] + [(nx - 1, j) for j in range(1, ny - 1)])
    tx = np.array([p[0] + 0.5 for p in per])
    ty = np.array([p[1] + 0.5 for p in per])
    dx, dy = tx - sx, ty - sy
    ix = np.full(len(per), int(math.floor(sx)))
    iy = np.full(len(per), int(math.floor(sy)))
    stepx = np.where(dx > 0, 1, -1)
    stepy = np.where(dy > 0, 1, -1)
    with np.errstate(divide="ignore", invalid="ignore"):
        tdx = np.where(dx != 0, np.abs(1.0 / dx), np.inf)
        tdy = np.where(dy != 0, np.abs(1.0 / dy), np.inf)
        tmx = np.where(dx > 0, (ix + 1 - sx) / dx, np.where(dx < 0, (ix - sx) / dx, np.inf))
        tmy = np.where(dy > 0, (iy + 1 - sy) / dy, np.where(dy < 0, (iy - sy) / dy, np.inf))
    ci = np.zeros(len(per), np.int64)  # x and y boundaries crossed so far
    cj = np.zeros(len(per), np.int64)
    seen = np.zeros((ny, nx), bool)
    active = np.ones(len(per), bool)
    for _ in range(2 * (nx + ny)):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        seen[iy[a], ix[a]] = True
        hit = occ[iy[a], ix[a]]
        active[a[hit]] = False
        a = a[~hit]
        # stop at the target perimeter cell
        done = (ix[a] == tx[a] - 0.5) & (iy[a] == ty[a] - 0.5)
        active[a[done]] = False
        a = a[~done]
        with np.errstate(invalid="ignore"):  # 0 * inf for an axis the ray does not move along
            cx = np.where(ci[a] == 0, tmx[a], tmx[a] + ci[a] * tdx[a])
            cy = np.where(cj[a] == 0, tmy[a], tmy[a] + cj[a] * tdy[a])
        go_x = cx < cy
        ax, ay = a[go_x], a[~go_x]
        ix[ax] += stepx[ax]
        ci[ax] += 1
        iy[ay] += stepy[ay]
        cj[ay] += 1
        out = (ix[a] < 0) | (ix[a] >= nx) | (iy[a] < 0) | (iy[a] >= ny)
        active[a[out]] = False
        ix[a[out]] = np.clip(ix[a[out]], 0, nx - 1)
        iy[a[out]] = np.clip(iy[a[out]], 0, ny - 1)
    return seen


def measurement_grid(occ: np.ndarray, rng: np.random.Generator, p_d=SENSOR["p_d"],
                     p_cl=SENSOR["p_cl"]):
    """(m_occ, m_free) float32 [ny*nx] for one cycle from a truth grid."""
    seen = raycast_observed(occ)
    det = np.where(occ, rng.random(occ.shape) < p_d, rng.random(occ.shape) < p_cl) & seen
    mo, mf = mass_levels(p_d, p_cl)
    m_occ = np.where(det, mo, 0.0).astype(np.float32).reshape(-1)
    m_free = np.where(seen & ~det, mf, 0.0).astype(np.float32).reshape(-1)
    return m_occ, m_free


def detection_grid(occ: np.ndarray, rng: np.random.Generator, p_d=SENSOR["p_d"],
                   p_cl=SENSOR["p_cl"]):
    """The observation of the particle PHD/MIB model (Sec. V.C) for one cycle, float32 [ny*nx]
    each: true / false positive probabilities p_tp = p_d, p_fp = p_cl where the cell is seen
    and 0.5 for both where it is not (no information), and the detection flag det (the same
    draws as measurement_grid)."""
    seen = raycast_observed(occ)
    det = np.where(occ, rng.random(occ.shape) < p_d, rng.random(occ.shape) < p_cl) & seen
    p_tp = np.where(seen, p_d, 0.5).astype(np.float32).reshape(-1)
    p_fp = np.where(seen, p_cl, 0.5).astype(np.float32).reshape(-1)
    return dict(p_tp=p_tp, p_fp=p_fp, det=det.astype(np.float32).reshape(-1))


def measurement_sequence(wl: dict, n_cycles: int, seed: int | None = None,
                         with_truth: bool = False, model: str = "ds"):
    """Measurement grids for cycles 1..n_cycles of the workload's scene: Dempster-Shafer masses
    (model "ds") or the detection observation of the particle PHD/MIB model (model "phd")."""
    seed = wl.get("seed", 0) if seed is None else seed
    scene = make_scene(wl, seed)
    out = []
    for k in range(1, n_cycles + 1):
        scene.advance()
        occ = scene.truth()
        rng = np.random.default_rng(np.random.SeedSequence([seed, k, 99]))
        if model == "phd":
            item = detection_grid(occ, rng)
        else:
            m_occ, m_free = measurement_grid(occ, rng)
            item = dict(m_occ=m_occ, m_free=m_free)
        if with_truth:
            vx, vy = scene.velocity_truth()
            item.update(occ=occ.reshape(-1), vx=vx.reshape(-1), vy=vy.reshape(-1))
        out.append(item)
    return out


def velocity_measurement(m_occ: np.ndarray, vx_true: np.ndarray, vy_true: np.ndarray,
                         rng: np.random.Generator, p_assoc=0.5, sd=1.0):
    """Doppler-like velocity evidence for detected cells: p_A, a measured velocity (truth +
    N(0, sd^2)) and its variance; zero association where nothing was detected."""
    det = m_occ > 0
    p_a = np.where(det, p_assoc, 0.0).astype(np.float32)
    mux = (vx_true + sd * rng.standard_normal(vx_true.shape)).astype(np.float32)
    muy = (vy_true + sd * rng.standard_normal(vy_true.shape)).astype(np.float32)
    var = np.full(vx_true.shape, sd * sd, np.float32)
    return dict(p_assoc=p_a, mu_vx=mux, mu_vy=muy, var_v=var)


def random_particles(nx: int, ny: int, cell: float, n: int, seed: int, spread: float = 1.0,
                     w_scale: float = 1e-3, out_frac: float = 0.01):
    """Arbitrary particle state (float32 dict) for edge-case and per-call tests: positions
    over the grid with a fraction just outside, velocities N(0, 5^2), weights U[0, 2 w_scale]
    with about 10 % exact zeros."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    W, H = nx * cell, ny * cell
    x = rng.uniform(-out_frac * W, (1 + out_frac) * W * spread, n)
    y = rng.uniform(-out_frac * H, (1 + out_frac) * H * spread, n)
    vx = 5.0 * rng.standard_normal(n)
    vy = 5.0 * rng.standard_normal(n)
    w = rng.uniform(0, 2 * w_scale, n)
    w[rng.random(n) < 0.1] = 0.0
    return {k: v.astype(np.float32) for k, v in dict(x=x, y=y, vx=vx, vy=vy, w=w).items()}


def random_measurement(C: int, seed: int, frac_occ=0.1, frac_free=0.5):
    """Arbitrary measurement grid: detections, free evidence and unobserved cells."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 88]))
    u = rng.random(C)
    mo, mf = mass_levels()
    m_occ = np.where(u < frac_occ, mo, 0.0)
    m_free = np.where((u >= frac_occ) & (u < frac_occ + frac_free), mf, 0.0)
    return dict(m_occ=m_occ.astype(np.float32), m_free=m_free.astype(np.float32))
