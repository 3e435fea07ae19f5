"""Test infrastructure: builds the library's kernels and C-ABI for the CPU, on the emulated HIP
subset of tests/emu/hip/hip_runtime.h, with AddressSanitizer (clang from the ROCm toolchain).

The sources are the library's own, with two mechanical rewrites the host compiler needs: the
device address-space attributes are dropped (the emulated memory is host memory, and the
sanitizer checks only default-address-space accesses), and a dynamic LDS declaration becomes a
pointer to the launch's LDS buffer, and every LDS array is refilled with a byte pattern when a
block starts (as uninitialised local variables are, by the compiler).  The velocity-evidence path is compiled in
(DOGM_EVIDENCE=1) and every array of a grid's arena is followed by a guard gap
(DOGM_ARENA_GAP) that the emulation poisons.

    python -m tests.emu.build_emu          # -> _build/emu/libdogm_emu.so
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
CSRC = os.path.join(ROOT, "paper_1605_02406_amd", "csrc")
EMU = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(ROOT, "_build", "emu")
LIB = os.path.join(OUT, "libdogm_emu.so")
SOURCES = ["k_particles.hip", "k_sort.hip", "k_cells.hip", "k_resample.hip", "k_sensor.hip",
           "dogm_api.cpp"]
HEADERS = ["dogm_internal.h", "launch.h"]
ARENA_GAP = 512

_AS = re.compile(r"__attribute__\(\(address_space\(\d+\)\)\)\s*")
_EXT_LDS = re.compile(r"extern\s+__shared__\s+([A-Za-z_][\w:]*)\s+(\w+)\[\];")
_LDS = re.compile(r"(?<!extern )__shared__\s+([A-Za-z_][\w:<>, ]*?)\s+(\w+)((?:\[[^\]]+\])+);")


def clangxx() -> str:
    for c in ("/opt/rocm/llvm/bin/clang++", "/opt/rocm/lib/llvm/bin/clang++"):
        if os.path.exists(c):
            return c
    raise RuntimeError("clang++ of the ROCm toolchain not found")


def asan_runtime() -> str:
    return subprocess.check_output([clangxx(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                                   text=True).strip()


def rewrite(text: str) -> str:
    text = _AS.sub("", text)
    text = _EXT_LDS.sub(r"\1* \2 = (\1*)::emu::dyn_lds();", text)
    # an LDS array holds no defined values when a block starts: refilled with a pattern once
    # per block, on the first thread that reaches the declaration
    return _LDS.sub(r"static \1 \2\3; ::emu::lds_fresh(\2, sizeof(\2));", text)


def _stage() -> str:
    src = os.path.join(OUT, "src")
    os.makedirs(src, exist_ok=True)
    for f in SOURCES + HEADERS:
        with open(os.path.join(CSRC, f)) as fh:
            text = rewrite(fh.read())
        dst = os.path.join(src, f if f.endswith((".h", ".cpp")) else f + ".cpp")
        old = open(dst).read() if os.path.exists(dst) else None
        if old != text:
            with open(dst, "w") as fh:
                fh.write(text)
    return src


def flags() -> list:
    return ["-std=c++17", "-O1", "-g", "-fPIC", "-ffp-contract=off", "-fsanitize=address",
            "-fno-omit-frame-pointer", "-shared-libsan", "-ftrivial-auto-var-init=pattern", "-DDOGM_EVIDENCE=1",
            f"-DDOGM_ARENA_GAP={ARENA_GAP}", "-Wno-unused-parameter",
            "-I", os.path.join(EMU), "-I", os.path.join(OUT, "src"), "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    src = _stage()
    os.makedirs(os.path.join(OUT, "obj"), exist_ok=True)
    units = [os.path.join(src, f if f.endswith(".cpp") else f + ".cpp") for f in SOURCES]
    units += [os.path.join(EMU, "emu_runtime.cpp"), os.path.join(EMU, "emu_guard.cpp")]

    def one(u):
        obj = os.path.join(OUT, "obj", os.path.basename(u) + ".o")
        if os.path.exists(obj) and os.path.getmtime(obj) >= max(
                os.path.getmtime(p) for p in [u, os.path.join(EMU, "hip", "hip_runtime.h")] +
                [os.path.join(src, h) for h in HEADERS]):
            return obj
        cmd = [clangxx(), *flags(), "-c", u, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"emulation build failed on {u}:\n{r.stderr[-4000:]}")
        if verbose:
            print("compiled", os.path.basename(u), flush=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(units), 6)) as ex:
        objs = list(ex.map(one, units))
    subprocess.check_call([clangxx(), "-shared", "-fsanitize=address", "-shared-libsan", *objs,
                           "-o", LIB])
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
