"""Test infrastructure: runs a scene through the CPU emulation of the library (built by
tests/emu/build_emu.py) call by call, each call checked against the oracle as on the GPU.  Run
in a process of its own with the AddressSanitizer runtime preloaded:

    LD_PRELOAD=$(clang++ -print-file-name=libclang_rt.asan-x86_64.so) \\
        python -m tests.emu.run_scene --workload small --cycles 3 --assoc
"""
from __future__ import annotations

import argparse
import ctypes as ct
import sys
import time

import numpy as np
import torch

from paper_1605_02406_amd import dogm, scenes
from tests.emu import build_emu


class HostStream:
    """The emulation runs every launch at once: its stream handle is null."""
    cuda_stream = 0


class HostMeas:
    """A measurement of host tensors in the shape of dogm.Meas."""

    def __init__(self, **t):
        self.t = {k: t.get(k) for k in ("m_occ", "m_free", "p_assoc", "mu_vx", "mu_vy", "var_v",
                                         "p_tp", "p_fp", "det")}
        self.c = dogm.CMeas(*[None if v is None else v.data_ptr() for v in self.t.values()])


def host_meas(m: dict) -> HostMeas:
    keep = ("m_occ", "m_free", "p_assoc", "mu_vx", "mu_vy", "var_v", "p_tp", "p_fp", "det")
    return HostMeas(**{k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).clone()
                       for k, v in m.items() if k in keep and v is not None})


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="small")
    ap.add_argument("--cycles", type=int, default=3)
    ap.add_argument("--n-pers", type=int, default=None)
    ap.add_argument("--n-born", type=int, default=None)
    ap.add_argument("--assoc", action="store_true", help="with velocity evidence (p_A > 0)")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--model", choices=("ds", "phd"), default="ds",
                    help="the Dempster-Shafer model of Sec. VI or the particle PHD/MIB model of Sec. V")
    args = ap.parse_args()

    dogm.LIB_PATH = build_emu.LIB  # the emulated build, loaded instead of the device library
    torch.cuda.synchronize = lambda *a, **k: None  # launches complete on return
    from tests import parity
    from tests.parity import PerCall

    # the checks read a grid's arrays before a call and compare after it: on the device those
    # reads are copies, here the arrays are host memory, so copy them
    parity.host = lambda t: np.array(t.cpu().numpy().view(np.uint32) if t.dtype == torch.int32
                                     else t.cpu().numpy())
    parity.u32 = lambda t: np.array(t.cpu().numpy().view(np.uint32))

    L = dogm.lib()
    L.emu_guard_arena.argtypes = [ct.c_void_p, ct.c_size_t]
    L.emu_guard_arena.restype = ct.c_int
    L.emu_counters.argtypes = [ct.POINTER(ct.c_uint64)]

    wl = scenes.WORKLOADS[args.workload]
    f = dict(scenes.FILTER)
    prec = dogm.PRECISION_FP64 if args.precision == "fp64" else dogm.PRECISION_FP32
    p = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], args.n_pers or wl["n_pers"],
                         wl["n_born"] if args.n_born is None else args.n_born, seed=0,
                         precision=prec,
                         model=dogm.MODEL_PHD_MIB if args.model == "phd" else dogm.MODEL_DS, **f)
    g = dogm.Grid(p, device="cpu", stream=HostStream())
    state = g.state
    g.state = lambda sorted_=False: {k: v.copy() for k, v in state(sorted_).items()}
    n = L.emu_guard_arena(ct.c_void_p(g.arena.data_ptr()), g.nbytes)
    if n < 0:
        print("[emu] arena arrays overlap or leave the arena", flush=True)
        return 2
    print(f"[emu] {args.workload} nu={p.n_pers} nb={p.n_born} assoc={args.assoc} "
          f"{n} arena arrays guarded", flush=True)
    seq = scenes.measurement_sequence(wl, args.cycles, with_truth=args.assoc, model=args.model)
    rng = np.random.default_rng(1)
    pc = PerCall(g)
    for k, m in enumerate(seq, start=1):
        m = dict(m)
        if args.assoc:
            m.update(scenes.velocity_measurement(m["m_occ"], m["vx"], m["vy"], rng))
        t0 = time.perf_counter()
        stats = pc.cycle(host_meas(m))
        worst = {kk: v for kk, v in stats.items() if isinstance(v, float)}
        print(f"[emu] cycle {k} checked in {time.perf_counter() - t0:.1f} s; largest relative "
              f"errors: " + ", ".join(f"{kk} {v:.1e}" for kk, v in sorted(worst.items())),
              flush=True)
    c = (ct.c_uint64 * 3)()
    L.emu_counters(c)
    print(f"[emu] launches {c[0]}, blocks {c[1]}, shuffles reading an inactive lane {c[2]}",
          flush=True)
    st = g.status()
    print(f"[emu] status word {st:#x}", flush=True)
    # a cell with new-born mass and no slot is reported, not an error (checked per call)
    return 0 if st & ~dogm.ST_NOCARRIER == 0 else 3


if __name__ == "__main__":
    sys.exit(main())
