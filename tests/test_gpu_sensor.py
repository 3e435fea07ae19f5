"""The device sensor (dogm_sensor_truth, dogm_sensor_scan) against the host scene generator:
the truth grid and the cells the ray cast observes must be bit-identical to Scene.truth() and
scenes.raycast_observed on the same scene; the evidence masses must equal a host evaluation of
the same Bernoulli draws (Philox4x32-10 words from the oracle's generator)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1605_02406_amd import dogm, scenes

pytestmark = pytest.mark.gpu

SENSOR_PURPOSE = 4


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()


def host_masses(occ, seen, seed, cycle, p_d, p_cl):
    """The detection draws of the device sensor, evaluated on the host."""
    mo, mf = scenes.mass_levels(p_d, p_cl)
    C = occ.size
    m_occ = np.zeros(C, np.float32)
    m_free = np.zeros(C, np.float32)
    for c in np.nonzero(seen.reshape(-1))[0]:
        u = oracle.uniform(int(oracle.philox([int(c), cycle, SENSOR_PURPOSE, 0], seed)[0]))
        det = u < (p_d if occ.reshape(-1)[c] else p_cl)
        m_occ[c] = np.float32(mo) if det else 0.0
        m_free[c] = 0.0 if det else np.float32(mf)
    return m_occ, m_free


SCENES = [("small", scenes.WORKLOADS["small"]), ("c512", scenes.WORKLOADS["c512"]),
          ("c1024", scenes.WORKLOADS["c1024"]),
          ("90x37", dict(nx=90, ny=37, cell=0.2, scene="boxes", n_boxes=6, clutter=0.02, seed=4)),
          ("1x50", dict(nx=1, ny=50, cell=0.2, scene="boxes", n_boxes=1, clutter=0.1, seed=5)),
          ("50x1", dict(nx=50, ny=1, cell=0.2, scene="boxes", n_boxes=1, clutter=0.1, seed=6)),
          ("2x2", dict(nx=2, ny=2, cell=0.2, scene="boxes", n_boxes=0, clutter=0.0, seed=7)),
          # wider than tall, 6 M cells and 10 000 rays of up to 5 000 steps
          ("3000x2000", dict(nx=3000, ny=2000, cell=0.1, scene="boxes", n_boxes=60, clutter=0.001,
                             seed=9))]


@pytest.mark.parametrize("name,wl", SCENES, ids=[s[0] for s in SCENES])
def test_device_sensor_equals_host_generator(name, wl):
    sc = scenes.make_scene(wl, wl.get("seed", 0))
    nx, ny = sc.nx, sc.ny
    dev = torch.device("cuda")
    static = torch.as_tensor(sc.static_mask().reshape(-1).astype(np.uint8), device=dev)
    occ = torch.zeros(nx * ny, dtype=torch.uint8, device=dev)
    seen = torch.zeros_like(occ)
    m_occ = torch.zeros(nx * ny, dtype=torch.float32, device=dev)
    m_free = torch.zeros_like(m_occ)
    for k in range(1, 4):
        sc.advance()
        print(f"[sensor] {name} cycle {k}", flush=True)
        rects = torch.as_tensor(sc.rects(), dtype=torch.float64, device=dev)
        dogm.sensor_truth(rects, static, nx, ny, sc.cell, occ)
        dogm.sensor_scan(occ, nx, ny, 0.9, 0.01, 11, k, seen, m_occ, m_free)
        torch.cuda.synchronize()
        truth = sc.truth()
        assert np.array_equal(occ.cpu().numpy().reshape(ny, nx) != 0, truth), "truth grid"
        ref_seen = scenes.raycast_observed(truth)
        assert np.array_equal(seen.cpu().numpy().reshape(ny, nx) != 0, ref_seen), "observed cells"
        if nx * ny <= 300_000:  # the host draws run cell by cell
            ho, hf = host_masses(truth, ref_seen, 11, k, 0.9, 0.01)
            assert np.array_equal(m_occ.cpu().numpy(), ho) and np.array_equal(m_free.cpu().numpy(), hf)
        assert float(m_occ.sum()) > 0 or not truth.any() or name in ("1x50", "50x1", "2x2")


def test_device_sensor_rejects_bad_arguments():
    dev = torch.device("cuda")
    occ = torch.zeros(16, dtype=torch.uint8, device=dev)
    with pytest.raises(dogm.DogmError):
        dogm.sensor_scan(occ, 4, 4, 0.01, 0.9, 1, 1, occ, None, None)  # p_D below p_cl
    with pytest.raises(dogm.DogmError):
        dogm.sensor_truth(None, None, 0, 4, 0.2, occ)


def test_truth_grid_edge_cases():
    """Rectangles partly or wholly outside the grid, infinite, empty, reversed, not a number,
    and bounds exactly on cell centres, against the per-cell definition."""
    inf, nan = float("inf"), float("nan")
    nx, ny, cell = 37, 23, 0.2
    rects = np.array([(-5.0, -5.0, 0.3, 0.3), (0.1, 0.1, 0.1, 0.1), (1e300, 0.0, 1e308, 5.0),
                      (-inf, 2.1, inf, 2.1), (nan, 0.0, 1.0, 1.0), (3.0, 1.0, 2.0, 4.0),
                      (0.5, 0.5, 1e308, 1e308), (-inf, -inf, -1.0, inf), (6.9, 4.5, 7.5, 4.5),
                      (2.3000000000000003, 0.7, 2.9, 1.3)], np.float64)
    static = (np.arange(nx * ny) % 11 == 0).astype(np.uint8)
    dev = torch.device("cuda")
    occ = torch.zeros(nx * ny, dtype=torch.uint8, device=dev)
    dogm.sensor_truth(torch.as_tensor(rects, device=dev), torch.as_tensor(static, device=dev),
                      nx, ny, cell, occ)
    torch.cuda.synchronize()
    xc = (np.arange(nx, dtype=np.float64) + 0.5) * cell
    yc = (np.arange(ny, dtype=np.float64) + 0.5) * cell
    ref = static.reshape(ny, nx) != 0
    for x0, y0, x1, y1 in rects:
        with np.errstate(invalid="ignore"):
            ref |= ((yc >= y0) & (yc <= y1))[:, None] & ((xc >= x0) & (xc <= x1))[None, :]
    assert np.array_equal(occ.cpu().numpy().reshape(ny, nx) != 0, ref)
