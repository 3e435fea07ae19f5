"""Test infrastructure: the device sensor (dogm_sensor_truth, dogm_sensor_scan) on the CPU
emulation of the library, against the host scene generator (truth grid and observed cells
bit-identical to Scene.truth() and scenes.raycast_observed).  Run with the AddressSanitizer
runtime preloaded, as tests/emu/run_scene.py."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_1605_02406_amd import dogm, scenes
from tests.emu import build_emu
from tests.emu.run_scene import HostStream

SCENES = [("small", scenes.WORKLOADS["small"], 3),
          ("c512", scenes.WORKLOADS["c512"], 1),
          ("90x37", dict(nx=90, ny=37, cell=0.2, scene="boxes", n_boxes=6, clutter=0.02, seed=4), 3),
          ("1x50", dict(nx=1, ny=50, cell=0.2, scene="boxes", n_boxes=1, clutter=0.1, seed=5), 2),
          ("50x1", dict(nx=50, ny=1, cell=0.2, scene="boxes", n_boxes=1, clutter=0.1, seed=6), 2),
          ("2x2", dict(nx=2, ny=2, cell=0.2, scene="boxes", n_boxes=0, clutter=0.0, seed=7), 1),
          # beyond the LDS bit mask (1.32 M cells): the rays read the occupancy bytes
          ("1200x1100", dict(nx=1200, ny=1100, cell=0.1, scene="boxes", n_boxes=40, clutter=0.002,
                             seed=8), 1)]


def truth_edge_cases(s) -> bool:
    """Rectangles partly or wholly outside the grid, infinite, empty, reversed, not a number,
    and bounds exactly on cell centres, against the per-cell definition in numpy."""
    inf, nan = float("inf"), float("nan")
    nx, ny, cell = 37, 23, 0.2
    rects = np.array([(-5.0, -5.0, 0.3, 0.3), (0.1, 0.1, 0.1, 0.1), (1e300, 0.0, 1e308, 5.0),
                      (-inf, 2.1, inf, 2.1), (nan, 0.0, 1.0, 1.0), (3.0, 1.0, 2.0, 4.0),
                      (0.5, 0.5, 1e308, 1e308), (-inf, -inf, -1.0, inf), (6.9, 4.5, 7.5, 4.5),
                      (2.3000000000000003, 0.7, 2.9, 1.3)], np.float64)
    static = (np.arange(nx * ny) % 11 == 0).astype(np.uint8)
    occ = torch.zeros(nx * ny, dtype=torch.uint8)
    dogm.sensor_truth(torch.as_tensor(rects), torch.as_tensor(static), nx, ny, cell, occ,
                      stream=s)
    xc = (np.arange(nx, dtype=np.float64) + 0.5) * cell
    yc = (np.arange(ny, dtype=np.float64) + 0.5) * cell
    ref = static.reshape(ny, nx) != 0
    for x0, y0, x1, y1 in rects:
        with np.errstate(invalid="ignore"):
            ref |= ((yc >= y0) & (yc <= y1))[:, None] & ((xc >= x0) & (xc <= x1))[None, :]
    ok = np.array_equal(occ.numpy().reshape(ny, nx) != 0, ref)
    print(f"[emu] truth edge cases {'equal' if ok else 'differ'} ({int(ref.sum())} occupied)",
          flush=True)
    return ok


def main() -> int:
    dogm.LIB_PATH = build_emu.LIB
    s = HostStream()
    if not truth_edge_cases(s):
        return 1
    for name, wl, cycles in SCENES:
        sc = scenes.make_scene(wl, wl.get("seed", 0))
        nx, ny = sc.nx, sc.ny
        static = torch.as_tensor(sc.static_mask().reshape(-1).astype(np.uint8))
        occ = torch.zeros(nx * ny, dtype=torch.uint8)
        seen = torch.zeros_like(occ)
        m_occ = torch.zeros(nx * ny, dtype=torch.float32)
        m_free = torch.zeros_like(m_occ)
        for k in range(1, cycles + 1):
            sc.advance()
            rects = torch.as_tensor(sc.rects(), dtype=torch.float64)
            dogm.sensor_truth(rects, static, nx, ny, sc.cell, occ, stream=s)
            dogm.sensor_scan(occ, nx, ny, 0.9, 0.01, 11, k, seen, m_occ, m_free, stream=s)
            truth = sc.truth()
            if not np.array_equal(occ.numpy().reshape(ny, nx) != 0, truth):
                print(f"[emu] {name} cycle {k}: truth grid differs", flush=True)
                return 1
            ref = scenes.raycast_observed(truth)
            got = seen.numpy().reshape(ny, nx) != 0
            if not np.array_equal(got, ref):
                print(f"[emu] {name} cycle {k}: observed cells differ in {int((got != ref).sum())}",
                      flush=True)
                return 1
            print(f"[emu] {name} cycle {k}: {int(ref.sum())} observed cells equal", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
