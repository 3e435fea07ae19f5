"""Launch plans (dogm_params.sort_passes, scan_parts) change no result: a grid stepped under
every plan the autotuner considers is bit-identical to the default plan, and the tuner returns
one of its candidates with a time for each."""
import pytest
import torch

from paper_1605_02406_amd import dogm, scenes, tune
from tests.parity import device_meas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()


@pytest.mark.parametrize("n", [64, 256])
def test_every_plan_gives_the_same_cycle(n):
    wl = scenes.batch_workload(n, seed=2)
    p = dogm.make_params(n, n, wl["cell"], wl["n_pers"], wl["n_born"], seed=4, **scenes.FILTER)
    seq = [device_meas(m) for m in scenes.measurement_sequence(wl, 3)]
    ref = dogm.Grid(p)
    grids = [dogm.Grid(tune.with_plan(p, plan)) for plan in tune.candidates(p)]
    assert len(grids) >= 2
    for meas in seq:
        ref.step(meas)
        for g in grids:
            g.step(meas)
    torch.cuda.synchronize()
    for g in grids:
        for name, t in ref.v.items():
            assert torch.equal(t, g.v[name]), name


def test_tuner_picks_a_candidate():
    wl = scenes.batch_workload(128, seed=1)
    p = dogm.make_params(128, 128, wl["cell"], wl["n_pers"], wl["n_born"], **scenes.FILTER)
    plan, report = tune.tune(p, warmup=2, cycles=3)
    assert plan in tune.candidates(p)
    assert len(report) == len(tune.candidates(p)) and all(v > 0 for v in report.values())


def test_blocks_adding_many_partials_match_the_scan():
    """More partial sums than a block reads in one round of loads (4 727 cell blocks of a
    1100 x 1100 grid; 5 120 resampling tiles of 2^22 + 2^18 particles): the cycle whose consumers
    add up the partials themselves equals, bit for bit, the one whose kernel scans them first,
    under both resampling kernels."""
    nx = 1100
    wl = dict(nx=nx, ny=nx, cell=0.2, n_pers=1 << 22, n_born=1 << 18, scene="boxes", n_boxes=40,
              clutter=0.01, seed=3)
    p = dogm.make_params(nx, nx, wl["cell"], wl["n_pers"], wl["n_born"], seed=5, **scenes.FILTER)
    seq = [device_meas(m) for m in scenes.measurement_sequence(wl, 2)]
    for res in (1, 2):
        grids = [dogm.Grid(tune.with_plan(p, dict(sort_passes=0, scan_parts=s, resample=res)))
                 for s in (1, 2)]
        for meas in seq:
            for g in grids:
                g.step(meas)
        torch.cuda.synchronize()
        for name, t in grids[0].v.items():
            assert torch.equal(t, grids[1].v[name]), (res, name)
        del grids


def test_grids_with_different_plans_share_a_batch():
    """One launch per kernel for grids whose launch plans differ (two and three sort passes, the
    partial sums scanned or added up by their consumers, both resampling kernels) gives every
    grid, bit for bit, the cycles it gets when stepped alone under its own plan."""
    plans = [dict(sort_passes=2, scan_parts=1, resample=1),
             dict(sort_passes=3, scan_parts=2, resample=2),
             dict(sort_passes=0, scan_parts=2, resample=1)]
    batched, alone, seqs = [], [], []
    for i, (n, plan) in enumerate(zip((128, 256, 200), plans)):
        wl = scenes.batch_workload(n, seed=i + 5)
        p = tune.with_plan(dogm.make_params(n, n, wl["cell"], wl["n_pers"], wl["n_born"],
                                            seed=9, grid_id=i, **scenes.FILTER), plan)
        batched.append(dogm.Grid(p))
        alone.append(dogm.Grid(p))
        seqs.append([device_meas(m) for m in scenes.measurement_sequence(wl, 3)])
    for k in range(3):
        dogm.step_batch(batched, [seq[k] for seq in seqs])
        for g, seq in zip(alone, seqs):
            g.step(seq[k])
    torch.cuda.synchronize()
    for gb, ga in zip(batched, alone):
        for name, t in ga.v.items():
            assert torch.equal(t, gb.v[name]), name
