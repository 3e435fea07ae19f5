"""GPU parity of every C-ABI call against the oracle (per-call, identical inputs), on scene
workloads and on edge cases.  See tests/parity.py for the tolerances."""
import numpy as np
import pytest
import torch

from paper_1605_02406_amd import dogm, scenes
from tests.parity import PerCall, device_meas, oracle_params, u32, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()  # fail loudly if the library is missing


def wl_params(wl, n_pers=None, n_born=None, seed=0, grid_id=0, **kw):
    f = dict(scenes.FILTER)
    f.update(kw)
    return dogm.make_params(wl["nx"], wl["ny"], wl["cell"], n_pers or wl["n_pers"],
                            wl["n_born"] if n_born is None else n_born, seed=seed,
                            grid_id=grid_id, **f)


def run_scene(name, cycles, n_pers=None, n_born=None, assoc=False, check_from=1, seed=0):
    wl = scenes.WORKLOADS[name]
    p = wl_params(wl, n_pers, n_born, seed=seed)
    g = dogm.Grid(p)
    seq = scenes.measurement_sequence(wl, cycles, with_truth=assoc)
    rng = np.random.default_rng(1)
    pc = PerCall(g)
    stats = []
    for k, m in enumerate(seq, start=1):
        m = dict(m)
        if assoc:
            m.update(scenes.velocity_measurement(m["m_occ"], m["vx"], m["vy"], rng))
        meas = device_meas(m)
        print(f"[parity] {name} cycle {k} nu={p.n_pers} nb={p.n_born} assoc={assoc}", flush=True)
        if k >= check_from:
            stats.append(pc.cycle(meas))
        else:
            g.step(meas)
    torch.cuda.synchronize()
    return g, stats


def test_small_scene_every_call_every_cycle():
    g, stats = run_scene("small", 6)
    worst = {k: max(s[k] for s in stats) for k in stats[0]}
    print("worst errors:", worst)
    assert g.status() & dogm.ST_NONFINITE == 0


@pytest.mark.skip(reason="velocity evidence is switched off: its first GPU run ended in a device "
                         "memory fault whose cause is not found yet (tests/test_emu.py runs the same "
                         "kernels on this scene clean and exact under AddressSanitizer)")
def test_small_scene_with_velocity_evidence():
    run_scene("small", 5, assoc=True)


def test_velocity_evidence_is_refused_before_any_launch():
    g, p = _fresh(8, 8, 100, 10)
    C = p.nx * p.ny
    m = scenes.random_measurement(C, 0)
    m.update(p_assoc=np.full(C, 0.5, np.float32), mu_vx=np.zeros(C, np.float32),
             mu_vy=np.zeros(C, np.float32), var_v=np.ones(C, np.float32))
    g.predict(); g.assign()
    with pytest.raises(dogm.DogmError) as e:
        g.update(device_meas(m))
    assert e.value.code == dogm.DOGM_ENOTIMPL and "disabled" in str(e.value)


@pytest.mark.parametrize("nu,nb", [(5000, 1), (12345, 777), (4096, 0), (1, 3), (70000, 4097)])
def test_ragged_sizes(nu, nb):
    run_scene("small", 3, n_pers=nu, n_born=nb)


def test_large_scene_512_full_size():
    """The 512x512 / 2^21 + 2^18 workload at full size, per-call parity on full arrays after a
    few cycles of warm-up (the launch configuration the benchmark times)."""
    g, stats = run_scene("c512", 4, check_from=3)
    print("c512 stats:", stats[-1])


def test_large_scene_1024_full_size():
    """The 1024x1024 / 2^23 + 2^20 workload at full size (two sort passes of 11 and 10 bits),
    per-call parity on full arrays in the second cycle."""
    g, stats = run_scene("c1024", 2, check_from=2)
    print("c1024 stats:", stats[-1])


def _fresh(nx, ny, nu, nb, **kw):
    p = dogm.make_params(nx, ny, 0.2, nu, nb, **kw)
    return dogm.Grid(p), p


def test_all_particles_in_one_cell_and_outside():
    g, p = _fresh(16, 16, 9000, 500, sigma_pos=0.0, sigma_vel=0.0)
    n = p.n_pers
    st = dict(x=np.full(n, 1.7, np.float32), y=np.full(n, 2.3, np.float32),
              vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
              w=np.full(n, 1e-4, np.float32))
    st["x"][::3] = -5.0  # a third leave the grid
    g.load_state(st)
    pc = PerCall(g)
    m = scenes.random_measurement(p.nx * p.ny, 3)
    m["m_occ"][:] = 0.9
    m["m_free"][:] = 0.0
    pc.cycle(device_meas(m))
    assert int((u32(g.v["cell_end"]) > u32(g.v["cell_start"])).sum()) == 1


def test_births_in_few_cells_span_many_tiles():
    """Births in three cells only (two of them in one wave of cells): each cell's slots span many
    new-born tiles, whose first-cell entries the wave writes together."""
    g, p = _fresh(32, 32, 20000, 6000, seed=4)
    C = p.nx * p.ny
    g.load_state(scenes.random_particles(p.nx, p.ny, 0.2, p.n_pers, 8))
    pc = PerCall(g)
    m = dict(m_occ=np.zeros(C), m_free=np.zeros(C))
    m["m_occ"][[3, 10, 700]] = 0.9
    pc.cycle(device_meas(m))
    off = u32(g.v["born_off"]).astype(np.int64)
    slots = off[1:] - off[:-1]
    assert int((slots > 0).sum()) == 3 and int(slots.max()) > 6 * 256  # more than 4 tiles


def test_vacuous_measurement_and_zero_weight():
    """Cycle 1 from the initial state (all weights 0) with an empty measurement: no mass,
    no births, the sorted state is kept by the resampling."""
    g, p = _fresh(20, 10, 3000, 400)
    C = p.nx * p.ny
    pc = PerCall(g)
    pc.cycle(device_meas(dict(m_occ=np.zeros(C), m_free=np.zeros(C))))
    assert int(g.v["S_fixed"].item()) == 0 and int(g.v["W_fixed"].item()) == 0
    assert np.all(u32(g.v["bkey"]) == C)


@pytest.mark.parametrize("nx,ny,nu,nb", [
    (40, 40, 20000, 3000),      # keys < 2^11: one pass of 11 bits
    (1500, 1500, 60000, 5000),  # keys < 2^22: two passes of 11 bits
    (2048, 2048, 60000, 5000),  # keys < 2^23: three passes of 8, 8 and 7 bits
])
def test_sort_plans(nx, ny, nu, nb):
    """Grids whose key range needs one, two and three radix passes with the widest digits,
    from arbitrary particle states, two cycles of per-call parity."""
    g, p = _fresh(nx, ny, nu, nb, seed=7, grid_id=3)
    g.load_state(scenes.random_particles(p.nx, p.ny, p.cell_size, p.n_pers, 7))
    pc = PerCall(g)
    for k in range(2):
        print(f"[parity] sort plan {nx}x{ny} cycle {k + 1}", flush=True)
        pc.cycle(device_meas(scenes.random_measurement(p.nx * p.ny, 20 + k)))


def test_random_states_and_measurements():
    for seed in range(3):
        g, p = _fresh(33, 27, 20000, 3000, seed=seed, grid_id=seed + 1)
        st = scenes.random_particles(p.nx, p.ny, p.cell_size, p.n_pers, seed)
        g.load_state(st)
        g.set_cycle(5 + seed)
        pc = PerCall(g)
        pc.cycle(device_meas(scenes.random_measurement(p.nx * p.ny, seed)))


def test_step_equals_call_sequence_and_is_deterministic():
    wl = scenes.WORKLOADS["small"]
    seq = scenes.measurement_sequence(wl, 4)
    outs = []
    for mode in ("calls", "step", "step"):
        g = dogm.Grid(wl_params(wl))
        for m in seq:
            meas = device_meas(m)
            if mode == "calls":
                g.predict(); g.assign(); g.update(meas); g.moments(); g.resample()
            else:
                g.step(meas)
        torch.cuda.synchronize()
        outs.append({k: host(v).copy() for k, v in g.v.items()})
    for other in outs[1:]:
        for k in outs[0]:
            assert np.array_equal(outs[0][k], other[k]), k


def test_batch_equals_single_grids():
    """Grids of different sizes stepped together are bit-identical to each stepped alone."""
    sizes = [(24, 24), (64, 64), (40, 17), (96, 96)]
    seqs, single = [], []
    for i, (nx, ny) in enumerate(sizes):
        wl = dict(nx=nx, ny=ny, cell=0.2, n_pers=8 * nx * ny, n_born=nx * ny, scene="boxes",
                  n_boxes=3, clutter=0.01, seed=i)
        seqs.append((wl, scenes.measurement_sequence(wl, 3, seed=i)))
    for i, (wl, seq) in enumerate(seqs):
        g = dogm.Grid(wl_params(wl, seed=11, grid_id=i))
        for m in seq:
            g.step(device_meas(m))
        torch.cuda.synchronize()
        single.append({k: host(v).copy() for k, v in g.v.items()})
    grids = [dogm.Grid(wl_params(wl, seed=11, grid_id=i)) for i, (wl, _) in enumerate(seqs)]
    for k in range(3):
        dogm.step_batch(grids, [device_meas(seq[k]) for _, seq in seqs])
    torch.cuda.synchronize()
    for g, ref in zip(grids, single):
        assert g.cycle == 4
        for k, v in g.v.items():
            assert np.array_equal(host(v), ref[k]), k


def test_batch_of_16_mixed_grids_at_full_size():
    """The 16-grid mix the benchmark's batched mode runs (128^2 to 768^2, 8 particles and one
    new-born slot per cell), two cycles in one batch, equals each grid stepped alone."""
    wls = [scenes.batch_workload(n, seed=i) for i, n in enumerate(scenes.BATCH_SIZES)]
    seqs = [[device_meas(m) for m in scenes.measurement_sequence(wl, 2)] for wl in wls]
    single = []
    for i, (wl, seq) in enumerate(zip(wls, seqs)):
        g = dogm.Grid(wl_params(wl, seed=i, grid_id=i))
        for m in seq:
            g.step(m)
        torch.cuda.synchronize()
        single.append({k: host(v).copy() for k, v in g.v.items()})
        del g
    grids = [dogm.Grid(wl_params(wl, seed=i, grid_id=i)) for i, wl in enumerate(wls)]
    for k in range(2):
        print(f"[parity] 16-grid batch cycle {k + 1}", flush=True)
        dogm.step_batch(grids, [seq[k] for seq in seqs])
    torch.cuda.synchronize()
    for i, (g, ref) in enumerate(zip(grids, single)):
        assert g.status() == 0
        for k, v in g.v.items():
            assert np.array_equal(host(v), ref[k]), (i, k)


def test_graph_replays_equal_eager_steps():
    """Cycles captured in HIP graphs (one graph per measurement) replay bit-identically to
    eager steps on a twin grid, with eager work and synchronisations between the replays."""
    wl = scenes.WORKLOADS["small"]
    seq = scenes.measurement_sequence(wl, 5)
    meas = [device_meas(m) for m in seq]
    eager, replayed = dogm.Grid(wl_params(wl)), dogm.Grid(wl_params(wl))
    eager.step(meas[0])
    replayed.step(meas[0])
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graphs = []
    for m in meas[1:]:
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            replayed.step(m)
        graphs.append(gr)
    for k, (gr, m) in enumerate(zip(graphs, meas[1:]), start=2):
        eager.step(m)
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        for name in ("x", "y", "vx", "vy", "w", "m_F", "m_O", "rho_b", "mean_x", "cell_start",
                     "perm", "bw", "W_fixed", "cycle"):
            assert np.array_equal(host(eager.v[name]), host(replayed.v[name])), (k, name)


def test_call_order_is_enforced():
    g, p = _fresh(8, 8, 100, 10)
    with pytest.raises(dogm.DogmError) as e:
        g.assign()
    assert e.value.code == dogm.DOGM_ESTATE
    g.predict()
    with pytest.raises(dogm.DogmError):
        g.predict()
    with pytest.raises(dogm.DogmError):
        g.resample()


def test_mass_bookkeeping_over_many_cycles():
    """Invariants over 15 cycles of the small scene: per-cell m_O + m_F <= 1, persistent weights
    sum to rho_p, the resampled total equals the joint weight."""
    wl = scenes.WORKLOADS["small"]
    g = dogm.Grid(wl_params(wl))
    C = wl["nx"] * wl["ny"]
    for k, m in enumerate(scenes.measurement_sequence(wl, 15), start=1):
        meas = device_meas(m)
        g.predict(); g.assign(); g.update(meas); g.moments()
        torch.cuda.synchronize()
        mo, mf = host(g.v["m_O"]).astype(float), host(g.v["m_F"]).astype(float)
        assert np.all(mo + mf <= 1 + 1e-6) and np.all(mo >= 0) and np.all(mf >= 0)
        start, end = u32(g.v["cell_start"]), u32(g.v["cell_end"])
        sw = host(g.v["sw"]).astype(float)
        cs = np.concatenate([[0], np.cumsum(sw)])
        per = cs[end] - cs[start]
        rp = host(g.v["rho_p"]).astype(float)
        has = host(g.v["sum_w"])[end > start] > 0
        np.testing.assert_allclose(per[end > start][has], rp[end > start][has], rtol=1e-5, atol=1e-9)
        joint = sw.sum() + host(g.v["bw"]).astype(float).sum()
        g.resample()
        torch.cuda.synchronize()
        W = int(g.v["W_fixed"].item()) * 2.0 ** -40
        assert W == pytest.approx(joint, rel=1e-6, abs=1e-9)
        assert host(g.v["w"]).astype(float).sum() == pytest.approx(W, rel=1e-5, abs=1e-9)
