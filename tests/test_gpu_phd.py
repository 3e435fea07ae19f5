"""GPU parity of the particle PHD/MIB model (Sec. V, p_A = 0) against the oracle, call by call:
the same harness and tolerances as the Dempster-Shafer model, with the detection observation
(true / false positive probabilities and detection flags) and births in every cell."""
import numpy as np
import pytest
import torch

from paper_1605_02406_amd import dogm, scenes
from tests.parity import PerCall, device_meas, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()


def phd_params(wl, n_pers=None, n_born=None, seed=0, grid_id=0):
    return dogm.make_params(wl["nx"], wl["ny"], wl["cell"], n_pers or wl["n_pers"],
                            wl["n_born"] if n_born is None else n_born, seed=seed,
                            grid_id=grid_id, model=dogm.MODEL_PHD_MIB, **scenes.FILTER)


def run_phd(name, cycles, check_from=1, n_pers=None, n_born=None):
    wl = scenes.WORKLOADS[name]
    g = dogm.Grid(phd_params(wl, n_pers, n_born))
    pc = PerCall(g)
    stats = []
    for k, m in enumerate(scenes.measurement_sequence(wl, cycles, model="phd"), start=1):
        print(f"[parity] phd {name} cycle {k}", flush=True)
        if k >= check_from:
            stats.append(pc.cycle(device_meas(m)))
        else:
            g.step(device_meas(m))
    torch.cuda.synchronize()
    return g, stats


def test_small_scene_every_call_every_cycle():
    g, stats = run_phd("small", 6)
    assert g.status() & dogm.ST_INTERNAL == 0
    # births in every cell that is not truncated: the new-born mass is spread over the grid
    assert int((host(g.v["rho_b"]) > 0).sum()) > 0.5 * g.C


@pytest.mark.parametrize("nu,nb", [(5000, 1), (12345, 777), (70000, 4097)])
def test_ragged_sizes(nu, nb):
    run_phd("small", 3, n_pers=nu, n_born=nb)


def test_large_scene_512_full_size():
    g, stats = run_phd("c512", 3, check_from=3)
    print("phd c512 stats:", stats[-1])


def test_batch_of_both_models_equals_single_grids():
    """Grids of the two models stepped in one batch (separate parameters per grid, one launch
    per kernel) are bit-identical to each stepped alone."""
    wl = scenes.WORKLOADS["small"]
    specs = [("phd", 0), ("ds", 1), ("phd", 2), ("ds", 3)]
    seqs = [[device_meas(m) for m in scenes.measurement_sequence(wl, 3, seed=i, model=kind)]
            for kind, i in specs]

    def params(kind, i):
        if kind == "phd":
            return phd_params(wl, seed=9, grid_id=i)
        return dogm.make_params(wl["nx"], wl["ny"], wl["cell"], wl["n_pers"], wl["n_born"],
                                seed=9, grid_id=i, **scenes.FILTER)

    single = []
    for (kind, i), seq in zip(specs, seqs):
        g = dogm.Grid(params(kind, i))
        for m in seq:
            g.step(m)
        torch.cuda.synchronize()
        single.append({k: host(v).copy() for k, v in g.v.items()})
    grids = [dogm.Grid(params(kind, i)) for kind, i in specs]
    for k in range(3):
        dogm.step_batch(grids, [seq[k] for seq in seqs])
    torch.cuda.synchronize()
    for j, (g, ref) in enumerate(zip(grids, single)):
        for k, v in g.v.items():
            assert np.array_equal(host(v), ref[k]), (j, k)


def test_measurement_of_the_other_model_is_refused():
    wl = scenes.WORKLOADS["small"]
    g = dogm.Grid(phd_params(wl))
    ds = device_meas(scenes.measurement_sequence(wl, 1)[0])
    g.predict()
    g.assign()
    with pytest.raises(dogm.DogmError) as e:
        g.update(ds)
    assert e.value.code == dogm.DOGM_EINVAL
