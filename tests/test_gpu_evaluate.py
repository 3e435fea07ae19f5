"""Filter quality on the synthetic lanes scene (Sec. VIII), through the GPU path: the paper's
qualitative findings on the birth probability p_B that the synthetic scene reproduces."""
import pytest
import torch

from paper_1605_02406_amd import dogm, evaluate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def results():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()
    return {pb: evaluate.evaluate(pb) for pb in (0.005, 0.02, 0.1)}


def test_velocity_of_moving_objects_is_estimated(results):
    r = results[0.02]
    assert r["samples"] >= 150
    assert r["velocity_mae_mps"] < 2.0          # objects move at 3 to 8 m/s


def test_new_born_particles_bias_the_velocity_towards_zero(results):
    # the birth velocity distribution has zero mean: more births, more bias (Sec. VIII.A)
    b = {pb: results[pb]["velocity_bias_along_motion_mps"] for pb in results}
    assert b[0.1] < b[0.02] - 0.2 and b[0.1] < b[0.005] - 0.2
    assert all(v < 0 for v in b.values())


def test_uncertainty_grows_with_the_birth_probability(results):
    sd = [results[pb]["velocity_sd_mps"] for pb in (0.005, 0.02, 0.1)]
    assert sd[0] < sd[1] < sd[2]


def test_estimates_are_consistent(results):
    # NEES of the x-velocity against the 95 % level of chi^2(1) (Sec. VIII.B)
    for pb, r in results.items():
        assert r["nees_frac_above_95pct"] < 0.15, pb


def test_moving_cells_separate_from_static_ones(results):
    # detected cells classified by the Mahalanobis distance of their velocity from zero
    # (Sec. VIII.C: a true positive rate near 99 % at 1 % false positives)
    for pb, r in results.items():
        assert r["roc_auc"] > 0.97, pb
    for pb in (0.005, 0.02):
        assert results[pb]["tpr_at_fpr_1pct"] > 0.9, pb
    # new-born particles blur the velocity of static cells: the separation is worst at high p_B
    assert results[0.1]["tpr_at_fpr_1pct"] < results[0.02]["tpr_at_fpr_1pct"]


@pytest.fixture(scope="module")
def approach():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()
    return {pb: evaluate.evaluate_approach(pb) for pb in (0.005, 0.1)}


def test_constant_velocity_model_lags_the_manoeuvres(approach):
    # an approaching object that accelerates, cruises and brakes (Sec. VIII.A): the estimate
    # trails the truth while the object accelerates and overshoots it while it brakes
    for pb, r in approach.items():
        ph = r["phases"]
        assert ph["accelerate"]["velocity_error_mean_mps"] < -0.5, pb
        assert ph["decelerate"]["velocity_error_mean_mps"] > ph["accelerate"]["velocity_error_mean_mps"] + 0.8, pb
    ph = approach[0.005]["phases"]
    assert ph["decelerate"]["velocity_error_mean_mps"] > 0.1
    assert abs(ph["stopped"]["velocity_error_mean_mps"]) < 0.3


def test_braking_nees_falls_with_the_birth_probability(approach):
    # Sec. VIII.B: a low p_B leaves the estimate least able to follow a strong deceleration
    lo = approach[0.005]["phases_detected_cells"]["decelerate"]["nees_mean"]
    hi = approach[0.1]["phases_detected_cells"]["decelerate"]["nees_mean"]
    assert lo > 2.0 * hi


def test_births_bias_the_cruising_object_towards_zero(approach):
    lo = approach[0.005]["phases"]["cruise"]["velocity_error_mean_mps"]
    hi = approach[0.1]["phases"]["cruise"]["velocity_error_mean_mps"]
    assert hi < lo - 0.3


@pytest.mark.parametrize("model", ["ds", "phd"])
def test_lanes_scene_every_call_against_the_oracle(model):
    """Per-call parity on the evaluation scene itself (320 x 160 cells, 2^19 + 2^16 particles):
    two cycles stepped, then three cycles checked call by call."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import numpy as np

    from paper_1605_02406_amd import scenes
    from tests.parity import PerCall, device_meas

    sc = evaluate.lanes_scene(seed=0)
    p = dogm.make_params(sc.nx, sc.ny, sc.cell, 1 << 19, 1 << 16, seed=0,
                         model=dogm.MODEL_PHD_MIB if model == "phd" else dogm.MODEL_DS,
                         **scenes.FILTER)
    g = dogm.Grid(p)
    pc = PerCall(g)
    for k in range(1, 6):
        sc.advance()
        occ = sc.truth()
        rng = np.random.default_rng(np.random.SeedSequence([0, k, 99]))
        if model == "phd":
            m = scenes.detection_grid(occ, rng)
        else:
            m_occ, m_free = scenes.measurement_grid(occ, rng)
            m = dict(m_occ=m_occ, m_free=m_free)
        print(f"[lanes] {model} cycle {k}", flush=True)
        if k <= 2:
            g.step(device_meas(m))
        else:
            pc.cycle(device_meas(m))
    assert g.status() & ~dogm.ST_NOCARRIER == 0
