"""Host logic of the synthetic input generator."""
import numpy as np

from paper_1605_02406_amd import scenes


def test_detection_grid_observation():
    """The particle PHD/MIB observation: informative probabilities where the sensor sees,
    none (p_tp = p_fp) where it does not, detections only in seen cells."""
    occ = np.zeros((20, 30), bool)
    occ[10, 20] = True           # an obstacle that hides the cells behind it
    m = scenes.detection_grid(occ, np.random.default_rng(0))
    seen = scenes.raycast_observed(occ).reshape(-1)
    assert np.all(m["p_tp"][seen] == np.float32(scenes.SENSOR["p_d"]))
    assert np.all(m["p_fp"][seen] == np.float32(scenes.SENSOR["p_cl"]))
    assert np.all(m["p_tp"][~seen] == m["p_fp"][~seen]) and (~seen).any()
    assert np.all(m["det"][~seen] == 0)
    assert set(np.unique(m["det"])) <= {0.0, 1.0}
