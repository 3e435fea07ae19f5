"""Test infrastructure: the library's multi-grid and allocation-free entry points on the CPU
emulation (see tests/emu/run_scene.py), under AddressSanitizer with guarded arenas:
  * dogm_step_batch on grids of different sizes, both precision modes and velocity evidence
    equals each grid stepped alone with dogm_step, bit for bit;
  * dogm_step_noalloc equals dogm_step bit for bit on two workloads in a row, the second
    smaller (the static scratch array keeps the first call's contents)."""
from __future__ import annotations

import ctypes as ct
import sys

import numpy as np

from paper_1605_02406_amd import dogm, scenes
from tests.emu import build_emu
from tests.emu.run_scene import HostStream, host_meas

S = HostStream()


def grid(L, wl, seed, grid_id, precision=None):
    kw = dict(scenes.FILTER)
    if precision is not None:
        kw["precision"] = precision
    p = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"], seed=seed,
                         grid_id=grid_id, **kw)
    g = dogm.Grid(p, device="cpu", stream=S)
    if L.emu_guard_arena(ct.c_void_p(g.arena.data_ptr()), g.nbytes) < 0:
        raise RuntimeError("arena arrays overlap")
    return g


def snapshot(g):
    return {k: np.array(v.numpy()) for k, v in g.v.items()}


def same(a: dict, b: dict, what: str) -> bool:
    for k in a:
        if not np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)):
            print(f"[emu] {what}: {k} differs", flush=True)
            return False
    return True


def batch(L) -> bool:
    specs = [((24, 24), None, False), ((64, 40), dogm.PRECISION_FP64, False),
             ((40, 17), None, False), ((48, 48), None, True), ((30, 30), None, True)]
    wls, seqs = [], []
    for i, ((nx, ny), prec, assoc) in enumerate(specs):
        wl = dict(nx=nx, ny=ny, cell=0.2, n_pers=8 * nx * ny, n_born=nx * ny, scene="boxes",
                  n_boxes=3, clutter=0.01, seed=i)
        seq = [dict(m) for m in scenes.measurement_sequence(wl, 3, seed=i, with_truth=assoc)]
        rng = np.random.default_rng(i)
        for m in seq:
            if assoc:
                m.update(scenes.velocity_measurement(m["m_occ"], m["vx"], m["vy"], rng))
        wls.append(wl)
        seqs.append([host_meas(m) for m in seq])
    single = []
    for i, (wl, (_, prec, _a)) in enumerate(zip(wls, specs)):
        g = grid(L, wl, 11, i, prec)
        for m in seqs[i]:
            g.step(m)
        single.append(snapshot(g))
    gs = [grid(L, wl, 11, i, prec) for i, (wl, (_, prec, _a)) in enumerate(zip(wls, specs))]
    for k in range(3):
        dogm.step_batch(gs, [seq[k] for seq in seqs], stream=S)
    ok = all(same(snapshot(g), ref, f"batch grid {i}") for i, (g, ref) in enumerate(zip(gs, single)))
    print(f"[emu] batch of {len(gs)} grids (two precisions, with and without evidence) "
          f"{'equals' if ok else 'differs from'} each grid alone", flush=True)
    return ok


def noalloc(L) -> bool:
    ok = True
    for i, (nx, ny, nu, nb) in enumerate([(64, 64, 32768, 8192), (40, 30, 5000, 777)]):
        wl = dict(nx=nx, ny=ny, cell=0.2, n_pers=nu, n_born=nb, scene="boxes", n_boxes=3,
                  clutter=0.01, seed=20 + i)
        seq = [host_meas(m) for m in scenes.measurement_sequence(wl, 3, seed=20 + i)]
        ref, got = grid(L, wl, 5, 0), grid(L, wl, 5, 0)
        for m in seq:
            ref.step(m)
            got.step_noalloc(m)
        ok &= same(snapshot(got), snapshot(ref), f"noalloc workload {i}")
    print(f"[emu] dogm_step_noalloc {'equals' if ok else 'differs from'} dogm_step on two "
          f"workloads in a row", flush=True)
    return ok


def main() -> int:
    dogm.LIB_PATH = build_emu.LIB
    L = dogm.lib()
    L.emu_guard_arena.argtypes = [ct.c_void_p, ct.c_size_t]
    L.emu_guard_arena.restype = ct.c_int
    ok = batch(L) & noalloc(L)
    c = (ct.c_uint64 * 3)()
    L.emu_counters.argtypes = [ct.POINTER(ct.c_uint64)]
    L.emu_counters(c)
    print(f"[emu] launches {c[0]}, blocks {c[1]}, shuffles reading an inactive lane {c[2]}",
          flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
