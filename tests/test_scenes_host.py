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


def test_no_box_blinds_the_sensor():
    """Every cycle of every workload's scene observes more than a thousand cells: no box drives
    over the sensor cell (which would stop every ray there)."""
    for name, n in (("small", 20), ("c512", 100), ("c1024", 50)):
        sc = scenes.make_scene(scenes.WORKLOADS[name])
        for k in range(1, n + 1):
            sc.advance()
            seen = int(scenes.raycast_observed(sc.truth()).sum())
            assert seen > 1000, (name, k, seen)


def test_box_reflects_off_the_sensor_keepout():
    """A box heading straight for the sensor turns back at the keep-out square and never
    covers the sensor cell."""
    sc = scenes.Scene(64, 64, 0.2, [scenes.Box(2.0, 6.4, 1.8, 1.0, 9.0, 0.0)], keepout=1.0)
    W, H = sc.size
    turned = False
    for _ in range(40):
        sc.advance()
        b = sc.boxes[0]
        assert abs(b.cx - W / 2) >= b.w / 2 + 1.0 - 1e-9 or abs(b.cy - H / 2) >= b.h / 2 + 1.0 - 1e-9
        assert not sc.truth()[32, 32]
        turned |= b.vx < 0 and b.cx > 3.0  # sent back on the sensor's side, not at the border
    assert turned
