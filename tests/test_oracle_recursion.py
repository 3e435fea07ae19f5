"""Whole-recursion pins of the oracle.

* Static world (the DS analogue of the paper's Proposition relating the PHD/MIB filter to the
  binary Bayes filter): with no motion, no noise, p_S = 1, p_B = 0, alpha = 1 and Bayesian
  measurement masses, every cell's occupied mass follows eq. (BBF_gen) exactly.
* Mass bookkeeping of every cycle on a synthetic scene: occupied mass = persistent + new-born
  particle weights = resampled weight total; m(O) + m(F) <= 1.
"""
import math

import numpy as np
import pytest

from paper_1605_02406_amd import scenes


def static_params(orc, nx, ny, nu):
    return orc.Params(nx, ny, 0.2, 0.1, 1.0, 0.0, 0.0, 0.0, 4.0, 1.0, nu, 64, seed=5)


def static_world(orc, seed, nx=8, ny=6, per_cell=5):
    rng = np.random.default_rng(seed)
    C = nx * ny
    m0 = rng.uniform(0.05, 0.95, C)
    cells = np.repeat(np.arange(C), per_cell)
    n = len(cells)
    frac = rng.dirichlet(np.ones(per_cell), C).reshape(-1)
    r = 0.2
    st = dict(x=(cells % nx + 0.5) * r, y=(cells // nx + 0.5) * r, vx=np.zeros(n), vy=np.zeros(n),
              w=m0[cells] * frac)
    return static_params(orc, nx, ny, n), st, m0


def bayes_meas(rng, C, p_tp=0.7, p_fp=0.2):
    det = rng.random(C) < 0.5
    alpha = np.where(det, p_tp / p_fp, (1 - p_tp) / (1 - p_fp))
    return dict(m_occ=alpha / (1 + alpha), m_free=1 / (1 + alpha)), alpha


def cell_mass(w, key, C):
    m = np.zeros(C + 1)
    np.add.at(m, key, w)
    return m[:C]


def test_static_world_is_binary_bayes_filter_without_resampling(orc):
    """Per step m_{k+1}(O) = alpha m_k / (alpha m_k + 1 - m_k), and over K steps
    logit m_K = logit m_0 + sum_k log alpha_k (closed form)."""
    p, st, m0 = static_world(orc, 1)
    C = p.C
    rng = np.random.default_rng(2)
    m_F = 1 - m0
    m = m0.copy()
    logit = np.log(m0 / (1 - m0))
    state = dict(st)
    for k in range(1, 9):
        meas, alpha = bayes_meas(rng, C)
        pred, key = orc.predict(p, k, state)
        perm, start, end = orc.assign(key, C)
        srt = {kk: pred[kk][perm] for kk in pred}
        cu = orc.cell_update(p, srt["w"], start, end, m_F, meas["m_occ"], meas["m_free"])
        w2, _, _ = orc.persistent_update(C, srt["w"], srt["vx"], srt["vy"], start, end, cu["rho_p"])
        srt["w"] = w2
        bbf = alpha * m / (alpha * m + 1 - m)
        assert np.allclose(cu["m_O"], bbf, rtol=1e-12, atol=0)
        assert np.allclose(cu["m_O"] + cu["m_F"], 1, atol=1e-12)
        assert np.all(cu["rho_b"] == 0)
        assert np.allclose(cell_mass(srt["w"], key[perm], C), bbf, rtol=1e-12)
        logit += np.log(alpha)
        m, m_F, state = cu["m_O"], cu["m_F"], srt
    assert np.allclose(np.log(m / (1 - m)), logit, rtol=1e-9, atol=1e-9)


def test_static_world_with_resampling(orc):
    """With systematic resampling each cell's mass moves by less than W/nu per cycle, and the
    update of every cycle is the binary Bayes filter of the resampled prior (truncated at 1),
    when the free mass entering the cycle is the Bayesian complement of that prior."""
    p, st, m0 = static_world(orc, 3, per_cell=40)
    C = p.C
    rng = np.random.default_rng(4)
    m_F = 1 - m0
    state = dict(st)
    for k in range(1, 7):
        meas, alpha = bayes_meas(rng, C)
        key0 = np.array([orc.cell_key_f64(p, x, y) for x, y in zip(state["x"], state["y"])])
        prior = np.minimum(cell_mass(state["w"], key0, C), 1.0)
        m_F = 1.0 - prior
        new, m_F, info = orc.cycle(p, k, state, m_F, meas)
        W = info["W_fixed"] * 2.0 ** -40
        bbf = alpha * prior / (alpha * prior + 1 - prior)
        assert np.allclose(info["m_O"], bbf, rtol=1e-12, atol=1e-15)
        key1 = np.array([orc.cell_key_f64(p, x, y) for x, y in zip(new["x"], new["y"])])
        post = cell_mass(new["w"], key1, C)
        assert np.all(np.abs(post - info["m_O"]) <= W / p.n_pers * (1 + 1e-9))
        state = new


@pytest.mark.parametrize("wl_name,assoc", [("small", False), ("small", True)])
def test_mass_bookkeeping_every_cycle(orc, wl_name, assoc):
    wl = dict(scenes.WORKLOADS[wl_name])
    wl["n_pers"], wl["n_born"] = 8192, 2048
    f = scenes.FILTER
    p = orc.Params(wl["nx"], wl["ny"], wl["cell"], f["dt"], f["p_s"], f["p_b"], f["sigma_pos"],
                   f["sigma_vel"], f["sigma_birth_vel"], f["alpha_free"], wl["n_pers"],
                   wl["n_born"], seed=0)
    C = p.C
    seq = scenes.measurement_sequence(wl, 6, with_truth=assoc)
    state = orc.init_state(p, p.n_pers)
    m_F = np.zeros(C)
    rng = np.random.default_rng(0)
    for k, meas in enumerate(seq, start=1):
        meas = dict(meas)
        if assoc:
            meas.update(scenes.velocity_measurement(meas["m_occ"], meas["vx"], meas["vy"], rng))
        new, m_F, info = orc.cycle(p, k, state, m_F, meas)
        srt, born = info["sorted"], info["born"]
        assert np.all(info["m_O"] + m_F <= 1 + 1e-12)
        assert np.all(info["rho_p"] >= -1e-15) and np.all(info["rho_b"] >= 0)
        # persistent weights per cell sum to rho_p wherever the cell had predicted mass
        pm = cell_mass(srt["w"], info["key"][info["perm"]], C)
        has = info["sum_w"] > 0
        assert np.allclose(pm[has], info["rho_p"][has], rtol=1e-12, atol=1e-15)
        # born weights per cell sum to rho_b wherever the cell received slots
        bm = cell_mass(born["w"][born["key"] < C], born["key"][born["key"] < C], C)
        n_c = np.diff(info["born_off"].astype(np.int64))
        assert np.allclose(bm[n_c > 0], info["rho_b"][n_c > 0], rtol=1e-12)
        # occupied mass = particle mass, up to births without a carrier (reported)
        lost = info["rho_b"][(n_c == 0)].sum()
        total = srt["w"].sum() + born["w"].sum()
        lost_p = info["rho_p"][~has].sum()  # persistent mass of cells without particles
        assert info["m_O"].sum() == pytest.approx(total + lost + lost_p, rel=1e-12)
        W = info["W_fixed"] * 2.0 ** -40
        assert W == pytest.approx(total, rel=1e-9)
        assert new["w"].sum() == pytest.approx(W, rel=1e-12)
        state = new
