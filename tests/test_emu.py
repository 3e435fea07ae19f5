"""The library's HIP kernels and C-ABI, compiled for the CPU on an emulation of the HIP subset
they use (tests/emu) and run under AddressSanitizer, call by call against the oracle.

This is where the velocity-evidence path (p_A > 0: Sec. VI, Alg. 4 and 5 with the likelihood,
Alg. 6 of the updated weights) runs end to end: on the device it is switched off until the
cause of a memory fault seen with it is shown.  Every array of the arena is followed by a
poisoned gap, every LDS array and uninitialised local variable starts from a byte pattern, and a
shuffle that reads an inactive lane is counted, so an out-of-range access or a read of
undefined data fails here."""
import os
import subprocess
import sys

import pytest

from tests.emu import build_emu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_env():
    try:
        build_emu.clangxx()
    except RuntimeError as e:
        pytest.skip(str(e))
    build_emu.build()
    env = dict(os.environ)
    env["LD_PRELOAD"] = build_emu.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    return env


def run(env, *args):
    r = subprocess.run([sys.executable, "-m", "tests.emu.run_scene", *args], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-6000:]
    assert "shuffles reading an inactive lane 0" in out
    return out


def test_small_scene_with_velocity_evidence(emu_env):
    run(emu_env, "--workload", "small", "--cycles", "3", "--assoc")


def test_ragged_sizes_with_velocity_evidence(emu_env):
    run(emu_env, "--workload", "small", "--cycles", "2", "--assoc", "--n-pers", "5000",
        "--n-born", "777")


def test_small_scene_without_evidence(emu_env):
    run(emu_env, "--workload", "small", "--cycles", "2")


def test_particle_phd_mib_model(emu_env):
    run(emu_env, "--workload", "small", "--cycles", "2", "--model", "phd")


def test_all_fp64_with_velocity_evidence(emu_env):
    run(emu_env, "--workload", "small", "--cycles", "2", "--assoc", "--precision", "fp64")


def test_device_sensor_equals_host_generator(emu_env):
    r = subprocess.run([sys.executable, "-m", "tests.emu.run_sensor"], cwd=ROOT, env=emu_env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-6000:]


def test_batched_and_allocation_free_cycles_equal_the_single_cycle(emu_env):
    r = subprocess.run([sys.executable, "-m", "tests.emu.run_modes"], cwd=ROOT, env=emu_env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-6000:]
    assert "shuffles reading an inactive lane 0" in out


def test_draws_piled_on_few_sources(emu_env):
    r = subprocess.run([sys.executable, "-m", "tests.emu.run_draws"], cwd=ROOT, env=emu_env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-6000:]
    assert "shuffles reading an inactive lane 0" in out
