"""Test infrastructure: emulated cycles whose resampling draws pile up on a few new-born
sources (births in one or a few cells, persistent weights near zero), so a wave's draws span
many LDS map windows and single sources receive thousands of draws; both resampling kernels,
each call checked against the oracle.  Run like tests/emu/run_scene.py, with the
AddressSanitizer runtime preloaded:

    python -m tests.emu.run_draws
"""
from __future__ import annotations

import ctypes as ct
import sys

import numpy as np
import torch

from paper_1605_02406_amd import dogm, scenes
from tests.emu import build_emu
from tests.emu.run_scene import HostStream, host_meas


def main() -> int:
    dogm.LIB_PATH = build_emu.LIB
    torch.cuda.synchronize = lambda *a, **k: None
    from tests import parity
    from tests.parity import PerCall
    parity.host = lambda t: np.array(t.cpu().numpy().view(np.uint32) if t.dtype == torch.int32
                                     else t.cpu().numpy())
    parity.u32 = lambda t: np.array(t.cpu().numpy().view(np.uint32))
    L = dogm.lib()
    L.emu_guard_arena.argtypes = [ct.c_void_p, ct.c_size_t]
    L.emu_guard_arena.restype = ct.c_int
    L.emu_counters.argtypes = [ct.POINTER(ct.c_uint64)]
    nx = ny = 32
    C = nx * ny
    # (new-born slots, cells with births): 300 slots in one cell (about 70 draws each, 17 map
    # windows per wave), 8 slots in one cell (2 500 draws each), 1 200 slots in three cells
    for nb, cells in ((300, [500]), (8, [77]), (1200, [3, 10, 700])):
        for mode in (1, 2):  # balanced, windowed
            p = dogm.make_params(nx, ny, 0.2, 20000, nb, seed=4, resample=mode)
            g = dogm.Grid(p, device="cpu", stream=HostStream())
            state = g.state
            g.state = lambda sorted_=False, state=state: {k: v.copy()
                                                          for k, v in state(sorted_).items()}
            if L.emu_guard_arena(ct.c_void_p(g.arena.data_ptr()), g.nbytes) < 0:
                print("[emu] arena arrays overlap or leave the arena", flush=True)
                return 2
            g.load_state(scenes.random_particles(nx, ny, 0.2, p.n_pers, 8, w_scale=1e-9))
            m = dict(m_occ=np.zeros(C), m_free=np.zeros(C))
            m["m_occ"][cells] = 0.9
            PerCall(g).cycle(host_meas(m))
            # the draws did concentrate: copies of one source share its position
            s = g.state()
            xy = np.stack([s["x"], s["y"]], axis=1)
            most = int(np.unique(xy, axis=0, return_counts=True)[1].max())
            st = g.status()
            print(f"[emu] nb={nb} births in {len(cells)} cell(s), resample mode {mode}: "
                  f"per-call parity ok, most draws of one source {most}, status {st:#x}",
                  flush=True)
            if st != 0 or (nb == 8 and most <= 1024):
                return 3
    c = (ct.c_uint64 * 3)()
    L.emu_counters(c)
    print(f"[emu] launches {c[0]}, blocks {c[1]}, shuffles reading an inactive lane {c[2]}",
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
