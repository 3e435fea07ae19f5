"""The all-FP64 precision mode (DOGM_PRECISION_FP64): every call compared with the oracle at the
tolerances of TOL64 in tests/parity.py (the FP32 mode's bar tightened by five orders), on the
64x64 scene, on ragged sizes and on the 1024x1024 / 2^23 + 2^20 workload at full size, where the
FP32 mode runs beside it at its own bar; a batch mixing both modes equals each grid alone."""
import numpy as np
import pytest
import torch

from paper_1605_02406_amd import dogm, scenes
from tests import parity
from tests.parity import PerCall, device_meas

pytestmark = pytest.mark.gpu

FP32, FP64 = dogm.PRECISION_FP32, dogm.PRECISION_FP64


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()


def run(wl, cycles, precision, check_from=1, n_pers=None, n_born=None, seed=0):
    p = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], n_pers or wl["n_pers"],
                         wl["n_born"] if n_born is None else n_born, seed=seed,
                         precision=precision, **scenes.FILTER)
    g = dogm.Grid(p)
    pc = PerCall(g)
    stats = None
    for k, m in enumerate(scenes.measurement_sequence(wl, cycles), start=1):
        print(f"[precision] {wl['nx']}x{wl['ny']} mode {precision} cycle {k}", flush=True)
        if k >= check_from:
            parity.P99.clear()
            stats = pc.cycle(device_meas(m))
        else:
            g.step(device_meas(m))
    torch.cuda.synchronize()
    assert g.status() & (dogm.ST_INTERNAL | dogm.ST_NONFINITE) == 0
    return g, stats, dict(parity.P99)


def test_fp64_small_scene_every_call_every_cycle():
    g, stats, _ = run(scenes.WORKLOADS["small"], 5, FP64)
    assert g.v["x"].dtype == torch.float64 and g.v["m_O"].dtype == torch.float64
    print("worst FP64 errors:", stats)


@pytest.mark.parametrize("nu,nb", [(5000, 1), (12345, 777), (70000, 4097)])
def test_fp64_ragged_sizes(nu, nb):
    run(scenes.WORKLOADS["small"], 3, FP64, n_pers=nu, n_born=nb)


def test_batch_of_both_precisions_equals_single_grids():
    wl = scenes.WORKLOADS["small"]
    seq = scenes.measurement_sequence(wl, 3)
    mk = lambda prec, gid: dogm.Grid(dogm.make_params(  # noqa: E731
        wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"], seed=1, grid_id=gid,
        precision=prec, **scenes.FILTER))
    alone = [mk(FP32, 0), mk(FP64, 1)]
    mixed = [mk(FP32, 0), mk(FP64, 1)]
    for m in seq:
        meas = device_meas(m)
        for g in alone:
            g.step(meas)
        dogm.step_batch(mixed, [meas, meas])
    torch.cuda.synchronize()
    for a, b in zip(alone, mixed):
        for name, t in a.v.items():
            assert torch.equal(t, b.v[name]), name


def test_precision_modes_at_1024_full_size():
    """The 1024x1024 / 2^23 + 2^20 workload in both modes, every call of the fourth cycle
    against the oracle at each mode's bar; the FP64 mode's errors must be far below FP32's."""
    wl = scenes.WORKLOADS["c1024"]
    _, s32, _ = run(wl, 4, FP32, check_from=4)
    _, s64, _ = run(wl, 4, FP64, check_from=4)
    for k in ("predict.x", "update.m_O", "update.rho_b", "update.w", "born.x", "moments.mean_x"):
        assert s64[k] < 1e-3 * max(s32[k], 1e-9), (k, s32[k], s64[k])
