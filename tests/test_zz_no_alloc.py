"""dogm_step_noalloc (the allocation-free cycle, include/dogm.h) against dogm_step: two grids
with the same parameters start from the same state and take the same measurements, one stepped
by each entry point; every array the grid exposes must be bit-identical after each cycle.  Two
workloads in a row, the second smaller, share the one static scratch array; a grid whose
scratch exceeds that array is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_1605_02406_amd import dogm, scenes
from tests.parity import device_meas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()


def _pair(wl, seed):
    p = dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"], seed=seed,
                         **scenes.FILTER)
    return dogm.Grid(p), dogm.Grid(p)


def _same(a: dogm.Grid, b: dogm.Grid, where: str):
    torch.cuda.synchronize()
    for name, t in a.v.items():
        assert torch.equal(t, b.v[name]), f"{where}: {name} differs"


def test_noalloc_step_equals_step():
    # a 256^2 grid with 2^19 + 2^16 particles, then the 64^2 workload with 2^15 + 2^13
    for name, wl, cycles in (("256^2", scenes.batch_workload(256, 3), 3),
                             ("64^2", scenes.WORKLOADS["small"], 4)):
        ref, got = _pair(wl, seed=7)
        seq = scenes.measurement_sequence(wl, cycles)
        for k, m in enumerate(seq, start=1):
            print(f"[noalloc] {name} cycle {k}", flush=True)
            meas = device_meas(m)
            ref.step(meas)
            got.step_noalloc(meas)
            _same(ref, got, f"{name} cycle {k}")
            assert got.cycle == ref.cycle == k + 1
        assert got.status() & dogm.ST_INTERNAL == 0


def test_noalloc_refuses_a_grid_beyond_the_static_array():
    p = dogm.make_params(64, 64, 0.2, 1 << 23, 1 << 10, **scenes.FILTER)
    g = dogm.Grid(p)
    m = device_meas(scenes.random_measurement(64 * 64, 1))
    with pytest.raises(dogm.DogmError) as e:
        g.step_noalloc(m)
    assert e.value.code == dogm.DOGM_ESIZE and "static array" in str(e.value)
    assert g.cycle == 1
    g.step(m)  # the grid is still usable through the arena's scratch
    torch.cuda.synchronize()
    assert g.cycle == 2
