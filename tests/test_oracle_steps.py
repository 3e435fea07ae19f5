"""Pins of the oracle's steps against what the paper and the mathematics fix: closed forms,
library routines, brute force and invariants.  None of these re-types the oracle's own
formula: each compares against an independent computation or a property."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_1605_02406_amd import scenes


def params(orc, nx=16, ny=12, nu=4096, nb=1024, **kw):
    d = dict(cell_size=0.2, dt=0.1, p_s=0.99, p_b=0.02, sigma_pos=0.1, sigma_vel=0.5,
             sigma_birth_vel=4.0, alpha_free=0.9, seed=3, grid_id=0)
    d.update(kw)
    return orc.Params(nx, ny, d.pop("cell_size"), d.pop("dt"), d.pop("p_s"), d.pop("p_b"),
                      d.pop("sigma_pos"), d.pop("sigma_vel"), d.pop("sigma_birth_vel"),
                      d.pop("alpha_free"), nu, nb, **d)


# ---------------------------------------------------------------------------------------
# a1 predict
# ---------------------------------------------------------------------------------------

def test_zero_noise_is_exact_cell_shift(orc):
    """Particles at cell centres with v = (a r/T, b r/T) land exactly (a, b) cells further,
    with weight p_S w; the predicted mass grid is the shifted grid times p_S."""
    p = params(orc, nx=20, ny=15, sigma_pos=0.0, sigma_vel=0.0)
    r, T = np.float32(p.cell_size), np.float32(p.dt)
    rng = np.random.default_rng(0)
    n = 3000
    ix, iy = rng.integers(0, p.nx, n), rng.integers(0, p.ny, n)
    a, b = rng.integers(-4, 5, n), rng.integers(-3, 4, n)
    st = dict(x=(ix + 0.5) * float(r), y=(iy + 0.5) * float(r), vx=a * float(r) / float(T),
              vy=b * float(r) / float(T), w=rng.uniform(0, 0.1, n))
    new, key = orc.predict(p, 1, st, noise=np.zeros((n, 4)))
    jx, jy = ix + a, iy + b
    inside = (jx >= 0) & (jx < p.nx) & (jy >= 0) & (jy < p.ny)
    C = p.C
    assert np.array_equal(key[inside], (jy * p.nx + jx)[inside])
    assert np.all(key[~inside] == C)
    assert np.allclose(new["w"][inside], float(np.float32(p.p_s)) * st["w"][inside], rtol=1e-15)
    assert np.all(new["w"][~inside] == 0)
    # mass grid: p_S times the old grid shifted by (a, b)
    old = np.zeros(C + 1)
    np.add.at(old, np.where(inside, jy * p.nx + jx, C), st["w"])
    pred = np.zeros(C + 1)
    np.add.at(pred, key, new["w"])
    assert np.allclose(pred[:C], float(np.float32(p.p_s)) * old[:C], rtol=1e-13, atol=0)


def test_predict_matches_cv_transition_matrix(orc):
    """x_{k+1} = F(T) x_k + G n with the constant-velocity matrix of eq. (process), computed
    as a matrix product."""
    p = params(orc)
    n = 500
    rng = np.random.default_rng(2)
    st = scenes.random_particles(p.nx, p.ny, p.cell_size, n, seed=4)
    noise = rng.standard_normal((n, 4))
    new, _ = orc.predict(p, 7, st, noise=noise)
    T = float(np.float32(p.dt))
    F = np.array([[1, 0, T, 0], [0, 1, 0, T], [0, 0, 1, 0], [0, 0, 0, 1]], float)
    G = np.diag([float(np.float32(p.sigma_pos))] * 2 + [float(np.float32(p.sigma_vel))] * 2)
    X = np.stack([st[k].astype(float) for k in ("x", "y", "vx", "vy")])
    ref = F @ X + G @ noise.T
    got = np.stack([new[k] for k in ("x", "y", "vx", "vy")])
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-12)


def test_predict_noise_scale_with_philox(orc):
    """With the oracle's own draws, (x' - x - T vx)/sigma_p etc. are N(0, 1) samples."""
    p = params(orc, nx=64, ny=64)
    n = 100_000
    st = dict(x=np.full(n, 6.4), y=np.full(n, 6.4), vx=np.full(n, 1.0), vy=np.full(n, -2.0),
              w=np.full(n, 1e-3))
    new, _ = orc.predict(p, 5, st)
    T, sp, sv = (float(np.float32(v)) for v in (p.dt, p.sigma_pos, p.sigma_vel))
    comps = [(new["x"] - 6.4 - T * 1.0) / sp, (new["y"] - 6.4 + T * 2.0) / sp,
             (new["vx"] - 1.0) / sv, (new["vy"] + 2.0) / sv]
    for z in comps:
        assert abs(z.mean()) < 5 / math.sqrt(n)
        assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)


def test_cell_key_f32_agrees_with_f64_away_from_edges(orc):
    p = params(orc, nx=37, ny=29)
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, p.nx * 0.2 + 1, 20000).astype(np.float32)
    y = rng.uniform(-1, p.ny * 0.2 + 1, 20000).astype(np.float32)
    k32 = orc.cell_keys_f32(p, x, y)
    k64 = np.array([orc.cell_key_f64(p, float(a), float(b)) for a, b in zip(x, y)])
    r = float(np.float32(p.cell_size))
    fx, fy = x.astype(float) / r, y.astype(float) / r
    edge = (np.abs(fx - np.round(fx)) < 1e-5) | (np.abs(fy - np.round(fy)) < 1e-5)
    assert np.array_equal(k32[~edge], k64[~edge])
    # outside the grid in either axis -> C
    assert np.all(k64[(fx < 0) | (fy < 0) | (fx >= p.nx) | (fy >= p.ny)] == p.C)


# ---------------------------------------------------------------------------------------
# a2 assign
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,C", [(0, 5), (1, 5), (257, 3), (5000, 97), (20000, 4096)])
def test_assign_is_numpy_stable_argsort(orc, n, C):
    rng = np.random.default_rng(n + C)
    key = rng.integers(0, C + 1, n).astype(np.uint32)
    perm, start, end = orc.assign(key, C)
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    counts = np.bincount(key, minlength=C + 1)
    assert np.array_equal(end.astype(int) - start.astype(int), counts[:C])
    assert np.array_equal(start, np.concatenate([[0], np.cumsum(counts[:C - 1])]).astype(np.uint32))
    if n <= 300:  # brute force: Python's sort is stable
        assert list(perm) == sorted(range(n), key=lambda i: int(key[i]))


def test_assign_rejects_bad_key(orc):
    with pytest.raises(ValueError):
        orc.assign(np.array([0, 7], np.uint32), 5)


# ---------------------------------------------------------------------------------------
# a3 Dempster combination and cell update
# ---------------------------------------------------------------------------------------

def dempster_powerset(m1, m2):
    """Dempster's rule by enumeration over 2^Omega with Omega = {O, F} as bitmasks
    (O = 1, F = 2, Omega = 3): conjunctive combination, then renormalise away the empty set."""
    acc = {0: 0.0, 1: 0.0, 2: 0.0, 3: 0.0}
    for (A, a), (B, b) in itertools.product(m1.items(), m2.items()):
        acc[A & B] += a * b
    k = acc.pop(0)
    return {A: v / (1 - k) for A, v in acc.items()}


def test_dempster_equals_powerset_enumeration(orc):
    rng = np.random.default_rng(3)
    for _ in range(3000):
        a = rng.dirichlet([1, 1, 1])
        b = rng.dirichlet([1, 1, 1])
        if rng.random() < 0.2:
            b = np.array([b[0] + b[2], b[1], 0.0])  # Bayesian measurement
        ref = dempster_powerset({1: a[0], 2: a[1], 3: a[2]}, {1: b[0], 2: b[1], 3: b[2]})
        o, f, conflict = orc.dempster(a[0], a[1], b[0], b[1])
        assert not conflict
        assert o == pytest.approx(ref[1], rel=1e-12, abs=1e-15)
        assert f == pytest.approx(ref[2], rel=1e-12, abs=1e-15)
        assert o + f <= 1 + 1e-12 and o >= 0 and f >= 0


def test_dempster_special_cases(orc):
    # vacuous measurement leaves the prediction unchanged
    o, f, _ = orc.dempster(0.3, 0.5, 0.0, 0.0)
    assert (o, f) == (pytest.approx(0.3, abs=1e-16), pytest.approx(0.5, abs=1e-16))
    # two Bayesian BBAs: the binary Bayes filter of eq. (BBF)
    for pz, pk in [(0.7, 0.2), (0.99, 0.5), (0.1, 0.9), (0.5, 0.5)]:
        o, f, _ = orc.dempster(pk, 1 - pk, pz, 1 - pz)
        bbf = pz * pk / (pz * pk + (1 - pz) * (1 - pk))
        assert o == pytest.approx(bbf, rel=1e-14) and o + f == pytest.approx(1, abs=1e-14)
    # total conflict keeps the prediction
    o, f, conflict = orc.dempster(1.0, 0.0, 0.0, 1.0)
    assert conflict and (o, f) == (1.0, 0.0)


def _cells_from_weights(orc, C, w_per_cell_lists):
    w, start, end = [], [], []
    for lst in w_per_cell_lists:
        start.append(len(w))
        w.extend(lst)
        end.append(len(w))
    return np.array(w, float), np.array(start, np.uint32), np.array(end, np.uint32)


def test_cell_update_closed_forms(orc):
    rng = np.random.default_rng(11)
    C = 400
    p = params(orc, nx=20, ny=20)
    lists = [list(rng.uniform(0, 0.25, rng.integers(0, 8))) for _ in range(C)]
    lists[0] = [0.7, 0.6]  # sum > 1: truncation
    w, start, end = _cells_from_weights(orc, C, lists)
    mfp = rng.uniform(0, 1, C)
    zo = np.where(rng.random(C) < 0.4, rng.uniform(0.5, 0.99, C), 0.0)
    zf = np.where(zo == 0, rng.uniform(0, 0.9, C) * (rng.random(C) < 0.7), 0.0)
    out = orc.cell_update(p, w, start, end, mfp, zo, zf)
    alpha, pB = float(np.float32(p.alpha_free)), float(np.float32(p.p_b))
    for c in range(C):
        s = sum(lists[c])
        assert out["sum_w"][c] == pytest.approx(s, rel=1e-14, abs=1e-300)
        mpo = min(s, 1.0)
        assert out["m_pO"][c] == pytest.approx(mpo, rel=1e-15)
        assert out["m_pF"][c] == pytest.approx(min(alpha * mfp[c], 1 - mpo), rel=1e-14, abs=1e-15)
        ref = dempster_powerset({1: mpo, 2: out["m_pF"][c], 3: 1 - mpo - out["m_pF"][c]},
                                {1: zo[c], 2: zf[c], 3: 1 - zo[c] - zf[c]})
        assert out["m_O"][c] == pytest.approx(ref[1], rel=1e-12, abs=1e-15)
        assert out["m_F"][c] == pytest.approx(ref[2], rel=1e-12, abs=1e-15)
        rb, rp, mo = out["rho_b"][c], out["rho_p"][c], out["m_O"][c]
        assert rb >= 0 and rp >= -1e-16 and rb + rp == pytest.approx(mo, abs=1e-15)
        assert rb + rp <= 1 + 1e-12
        if zo[c] == 0:
            assert rb == 0  # new-born mass only where the measurement reports occupancy
        elif mpo == 0:
            assert rb == pytest.approx(mo, rel=1e-15)
        elif mo > 0 and rp > 0:
            # eq. (DS_relation_masses) with the predicted occupied mass
            assert rb / rp == pytest.approx(pB * (1 - mpo) / mpo, rel=1e-11)
        assert out["pign"][c] == pytest.approx(mo + 0.5 * (1 - mo - out["m_F"][c]), abs=1e-15)
    assert out["m_pO"][0] == 1.0


def test_cell_update_without_birth(orc):
    p = params(orc, nx=10, ny=10, p_b=0.0)
    rng = np.random.default_rng(1)
    lists = [list(rng.uniform(0, 0.2, rng.integers(0, 6))) for _ in range(100)]
    w, start, end = _cells_from_weights(orc, 100, lists)
    zo = np.where(rng.random(100) < 0.5, 0.9, 0.0)
    out = orc.cell_update(p, w, start, end, np.zeros(100), zo, np.zeros(100))
    assert np.all(out["rho_b"] == 0) and np.allclose(out["rho_p"], out["m_O"])


# ---------------------------------------------------------------------------------------
# a4 persistent update
# ---------------------------------------------------------------------------------------

def _random_cells(rng, C, maxn=10):
    lists = [rng.uniform(0, 0.2, rng.integers(0, maxn)) for _ in range(C)]
    start = np.cumsum([0] + [len(l) for l in lists[:-1]]).astype(np.uint32)
    end = np.cumsum([len(l) for l in lists]).astype(np.uint32)
    return np.concatenate(lists), start, end


def test_persistent_update_mass_conservation(orc):
    rng = np.random.default_rng(5)
    C = 300
    w, start, end = _random_cells(rng, C)
    n = len(w)
    vx, vy = rng.normal(0, 3, n), rng.normal(0, 3, n)
    rho_p = rng.uniform(0, 1, C)
    for kw in [dict(), dict(p_assoc=rng.uniform(0, 1, C), mu_vx=rng.normal(0, 3, C),
                            mu_vy=rng.normal(0, 3, C), var_v=rng.uniform(0.5, 4, C))]:
        w2, mu_A, mu_UA = orc.persistent_update(C, w, vx, vy, start, end, rho_p, **kw)
        for c in range(C):
            s = w2[start[c]:end[c]].sum()
            if end[c] > start[c] and w[start[c]:end[c]].sum() > 0:
                assert s == pytest.approx(rho_p[c], rel=1e-12)
        assert np.all(w2 >= 0)


def test_persistent_update_association_limits(orc):
    rng = np.random.default_rng(6)
    C = 50
    w, start, end = _random_cells(rng, C, maxn=12)
    n = len(w)
    vx, vy = rng.normal(0, 2, n), rng.normal(0, 2, n)
    rho_p = rng.uniform(0.1, 1, C)
    mux, muy, var = rng.normal(0, 2, C), rng.normal(0, 2, C), rng.uniform(1, 3, C)
    cell = np.repeat(np.arange(C), (end - start).astype(int))
    # p_A = 0: the likelihood is ignored, w' proportional to w
    w0, _, _ = orc.persistent_update(C, w, vx, vy, start, end, rho_p, np.zeros(C), mux, muy, var)
    wn, _, _ = orc.persistent_update(C, w, vx, vy, start, end, rho_p)
    assert np.allclose(w0, wn, rtol=1e-14)
    # p_A = 1: w' proportional to g(z|x) w within each cell
    w1, _, _ = orc.persistent_update(C, w, vx, vy, start, end, rho_p, np.ones(C), mux, muy, var)
    g = np.exp(-((vx - mux[cell]) ** 2 + (vy - muy[cell]) ** 2) / (2 * var[cell]))
    for c in range(C):
        sl = slice(start[c], end[c])
        if end[c] > start[c] and (g[sl] * w[sl]).sum() > 0:
            ref = rho_p[c] * g[sl] * w[sl] / (g[sl] * w[sl]).sum()
            assert np.allclose(w1[sl], ref, rtol=1e-12, atol=1e-300)
    # a likelihood that is constant in the cell makes the result independent of p_A
    same = dict(mu_vx=np.zeros(C), mu_vy=np.zeros(C), var_v=np.ones(C))
    vz = np.zeros(n)
    wa, _, _ = orc.persistent_update(C, w, vz, vz, start, end, rho_p, np.full(C, 0.3), **same)
    wb, _, _ = orc.persistent_update(C, w, vz, vz, start, end, rho_p, np.full(C, 0.9), **same)
    assert np.allclose(wa, wb, rtol=1e-14) and np.allclose(wa, wn, rtol=1e-14)


# ---------------------------------------------------------------------------------------
# a5 new-born particles
# ---------------------------------------------------------------------------------------

def test_born_alloc_proportional(orc):
    rng = np.random.default_rng(8)
    for C, nb in [(1, 7), (50, 1000), (4096, 8192), (10000, 333)]:
        rho_b = np.where(rng.random(C) < 0.3, rng.uniform(0, 0.5, C), 0.0)
        off, S = orc.born_alloc(C, nb, rho_b)
        assert S == sum(orc.fixed40(v) for v in rho_b)
        if C == 1:
            rho_b[:] = 0.4
            off, S = orc.born_alloc(C, nb, rho_b)
        n = np.diff(off.astype(np.int64))
        assert n.sum() == nb and np.all(n >= 0) and off[0] == 0 and off[-1] == nb
        q = np.array([orc.fixed40(v) for v in rho_b], dtype=object)
        for c in range(C):
            exact = Fraction(int(q[c]) * nb, S)  # nu_b rho_b / S in exact rationals
            assert abs(Fraction(int(n[c])) - exact) < 1
    off, S = orc.born_alloc(10, 100, np.zeros(10))
    assert S == 0 and np.all(off == 0)


def test_born_alloc_every_slot_lies_in_a_cell_with_mass(orc):
    """Cells after the last cell with new-born mass own no slot, and every slot belongs to a cell
    with mass (eq. (weights_unassociated) needs rho_b > 0 wherever n_c > 0).  With nu_b = 777 and
    S = 248694042651024 (units of 2^-40) the FP64 quotient fl(fl(S nu_b) / S) is just below 777,
    so the share of a trailing cell must come from its definition (all mass before it), not
    from that rounding."""
    rng = np.random.default_rng(9)
    cases = [(777, 248694042651024)]
    cases += [(int(rng.integers(2, 5000)), int(rng.integers(1 << 41, 1 << 47))) for _ in range(60)]
    for nb, S in cases:
        n_mass = 2 * -(-S // (1 << 40)) + 5  # cells holding S with masses of about 1/2
        # n_mass near-equal parts of S, each moved by a random amount
        base = np.full(n_mass, S // n_mass, np.int64)
        base[: S - int(base.sum())] += 1
        jig = rng.integers(0, (S // n_mass) // 4, n_mass // 2)
        base[: n_mass // 2] -= jig
        base[n_mass // 2: 2 * (n_mass // 2)] += jig
        q = base
        assert q.sum() == S and q.max() < (1 << 40)
        C = n_mass + 30
        rho_b = np.zeros(C)
        rho_b[:n_mass] = q.astype(np.float64) * 2.0 ** -40  # exact: q < 2^40
        off, S_got = orc.born_alloc(C, nb, rho_b)
        assert S_got == S
        assert np.all(off[n_mass:] == nb), (nb, S)
        cell_of_slot = np.searchsorted(off, np.arange(nb), side="right") - 1
        assert np.all(rho_b[cell_of_slot] > 0), (nb, S)


def test_born_init_properties(orc):
    p = params(orc, nx=12, ny=9, nb=6000, seed=21)
    C = p.C
    rng = np.random.default_rng(2)
    rho_b = np.where(rng.random(C) < 0.5, rng.uniform(0, 0.3, C), 0.0)
    rho_b[0] = 0.25
    off, S = orc.born_alloc(C, p.n_born, rho_b)
    pa = np.where(rng.random(C) < 0.5, rng.uniform(0, 1, C), 0.0)
    mux, muy = rng.normal(0, 5, C), rng.normal(0, 5, C)
    var = rng.uniform(0.5, 2, C)
    b = orc.born_init(p, 4, off, rho_b, pa, mux, muy, var)
    r = float(np.float32(p.cell_size))
    n = np.diff(off.astype(int))
    for c in range(C):
        sl = slice(off[c], off[c + 1])
        if n[c] == 0:
            continue
        assert np.all(b["key"][sl] == c)
        assert b["w"][sl].sum() == pytest.approx(rho_b[c], rel=1e-12)
        na = int(b["assoc"][sl].sum())
        assert na == math.floor(pa[c] * n[c] + 0.5)
        if 0 < na < n[c]:  # the associated set carries p_A of the new-born mass
            assert b["w"][sl][b["assoc"][sl] == 1].sum() == pytest.approx(pa[c] * rho_b[c], rel=1e-12)
        ix, iy = c % p.nx, c // p.nx
        assert np.all((b["x"][sl] >= ix * r) & (b["x"][sl] <= (ix + 1) * r))
        assert np.all((b["y"][sl] >= iy * r) & (b["y"][sl] <= (iy + 1) * r))
    # unassociated velocities ~ N(0, sigma_B^2); associated ~ N(mu_z, var_z)
    un = b["assoc"] == 0
    sB = float(np.float32(p.sigma_birth_vel))
    z = np.concatenate([b["vx"][un], b["vy"][un]]) / sB
    assert abs(z.mean()) < 5 / math.sqrt(len(z)) and abs(z.var() - 1) < 5 * math.sqrt(2 / len(z))
    a = b["assoc"] == 1
    za = (b["vx"][a] - mux[b["key"][a]]) / np.sqrt(var[b["key"][a]])
    assert abs(za.mean()) < 5 / math.sqrt(len(za)) and abs(za.var() - 1) < 5 * math.sqrt(2 / len(za))


def test_born_init_without_birth(orc):
    p = params(orc, nx=4, ny=4, nb=64)
    off, S = orc.born_alloc(p.C, p.n_born, np.zeros(p.C))
    b = orc.born_init(p, 1, off, np.zeros(p.C))
    assert np.all(b["w"] == 0) and np.all(b["key"] == p.C)


# ---------------------------------------------------------------------------------------
# a6 moments
# ---------------------------------------------------------------------------------------

def test_moments_match_numpy_weighted_statistics(orc):
    rng = np.random.default_rng(12)
    C = 200
    w, start, end = _random_cells(rng, C, maxn=15)
    n = len(w)
    vx, vy = rng.normal(3, 4, n), rng.normal(-2, 1, n)
    S0 = np.array([w[start[c]:end[c]].sum() for c in range(C)])
    m = orc.moments(C, w, vx, vy, start, end, S0)  # rho_p equal to the weight sum
    for c in range(C):
        sl = slice(start[c], end[c])
        if end[c] - start[c] < 1 or S0[c] == 0:
            assert m["flag"][c] == 0 and m["mean_x"][c] == 0
            continue
        assert m["mean_x"][c] == pytest.approx(np.average(vx[sl], weights=w[sl]), rel=1e-12, abs=1e-12)
        assert m["mean_y"][c] == pytest.approx(np.average(vy[sl], weights=w[sl]), rel=1e-12, abs=1e-12)
        if end[c] - start[c] >= 2:
            cov = np.cov(vx[sl], vy[sl], aweights=w[sl], bias=True)
            assert m["var_x"][c] == pytest.approx(cov[0, 0], rel=1e-9, abs=1e-10)
            assert m["var_y"][c] == pytest.approx(cov[1, 1], rel=1e-9, abs=1e-10)
            assert m["cov_xy"][c] == pytest.approx(cov[0, 1], rel=1e-9, abs=1e-10)
    # normalisation by rho_p as printed: doubling rho_p halves the mean
    m2 = orc.moments(C, w, vx, vy, start, end, 2 * S0)
    ok = m["flag"] == 1
    assert np.allclose(m2["mean_x"][ok], m["mean_x"][ok] / 2, rtol=1e-13)


def test_moments_constant_velocity(orc):
    C = 30
    rng = np.random.default_rng(1)
    w, start, end = _random_cells(rng, C, maxn=9)
    cell = np.repeat(np.arange(C), (end - start).astype(int))
    v = rng.normal(0, 10, (C, 2))
    S0 = np.array([w[start[c]:end[c]].sum() for c in range(C)])
    m = orc.moments(C, w, v[cell, 0], v[cell, 1], start, end, S0)
    ok = m["flag"] == 1
    assert np.allclose(m["mean_x"][ok], v[ok, 0], rtol=1e-13)
    assert np.allclose(m["var_x"][ok], 0, atol=1e-12 * (1 + v[ok, 0] ** 2))
    assert np.allclose(m["cov_xy"][ok], 0, atol=1e-12 * (1 + np.abs(v[ok]).prod(1)))


# ---------------------------------------------------------------------------------------
# a7 resampling
# ---------------------------------------------------------------------------------------

def test_resample_systematic_properties(orc):
    rng = np.random.default_rng(4)
    for nu, nb in [(1, 0), (10, 3), (1000, 100), (4096, 1024), (30000, 7000)]:
        wp = np.where(rng.random(nu) < 0.8, rng.uniform(0, 1e-2, nu), 0.0)
        wb = np.where(rng.random(nb) < 0.8, rng.uniform(0, 1e-2, nb), 0.0)
        if nu == 1:
            wp[:] = 0.3
        U = orc.uniform(int(rng.integers(0, 2 ** 32)))
        idx, W = orc.resample_indices(wp, wb, U)
        q = np.array([orc.fixed40(v) for v in np.concatenate([wp, wb])], dtype=np.int64)
        assert W == int(q.sum())
        assert np.all(np.diff(idx) >= 0)  # systematic draws give sorted indices
        assert np.all(q[idx] > 0)  # zero-weight particles are never drawn
        counts = np.bincount(idx, minlength=nu + nb)
        exact = q.astype(object) * nu  # expected counts nu q_i / W, as exact rationals
        for i in np.nonzero(q)[0]:
            e = Fraction(int(exact[i]), W)
            assert math.floor(e) - 1 <= counts[i] <= math.ceil(e) + 1
            assert abs(counts[i] - e) < 1 + 1e-9  # floor or ceil of nu q_i / W
        ow = orc.resample_weight(W, nu)
        assert ow * nu == pytest.approx(W * 2.0 ** -40, rel=1e-15)


def test_resample_unbiased_over_offset(orc):
    """Sweeping U over [0, 1): the expected number of copies of particle i is nu q_i / W
    (exact rationals, brute force over the breakpoints of the piecewise-constant map)."""
    rng = np.random.default_rng(7)
    nu, nb = 7, 3
    wp = rng.integers(1, 50, nu) * 2.0 ** -10
    wb = rng.integers(0, 50, nb) * 2.0 ** -10
    q = np.array([orc.fixed40(v) for v in np.concatenate([wp, wb])], dtype=np.int64)
    W = int(q.sum())
    F = np.cumsum(q)
    # breakpoints of U where some draw (j + U) W / nu crosses an F_i
    bps = sorted({0.0, 1.0} | {float(Fraction(int(f) * nu, W) - j) for f in F for j in range(nu)
                               if 0 < Fraction(int(f) * nu, W) - j < 1})
    expect = np.zeros(nu + nb)
    for a, b in zip(bps[:-1], bps[1:]):
        idx, _ = orc.resample_indices(wp, wb, (a + b) / 2)
        expect += (b - a) * np.bincount(idx, minlength=nu + nb)
    ref = q * nu / W
    assert np.allclose(expect, ref, rtol=1e-12, atol=1e-12)


def test_resample_zero_total_keeps_state(orc):
    idx, W = orc.resample_indices(np.zeros(5), np.zeros(2), 0.5)
    assert W == 0 and list(idx) == [0, 1, 2, 3, 4]


def test_resample_draw_lies_in_chosen_interval(orc):
    """Each systematic draw u_j = (j + U) d, d = W / nu, lies in the half-open CDF interval
    [F_{i-1}, F_i) of the particle it selects (exact rationals).  Includes draws that hit a
    boundary exactly: those belong to the next particle."""
    # w = (1/4, 3/4), nu = 2, U = 1/2: u_0 = W/4 = F_0 exactly -> particle 1
    idx, W = orc.resample_indices(np.array([0.25, 0.75]), np.zeros(0), 0.5)
    assert list(idx) == [1, 1]
    # equal weights, U = 1/2: draws at (j + 1/2) W / nu; with nu = 2 N every other draw
    # sits exactly on a boundary
    N = 8
    idx, W = orc.resample_indices(np.full(N, 1.0 / 16), np.zeros(0), 0.5)
    assert list(idx) == [0, 1, 2, 3, 4, 5, 6, 7]
    rng = np.random.default_rng(17)
    for trial in range(40):
        # nu a power of two: the spacing W / nu and every draw are exact in FP64, so the
        # oracle's draws equal the exact rationals below
        nu, nb = 2 ** int(rng.integers(0, 6)), int(rng.integers(0, 10))
        wp = rng.integers(0, 9, nu) * 2.0 ** -6
        wb = rng.integers(0, 9, nb) * 2.0 ** -6
        if wp.sum() + wb.sum() == 0:
            continue
        U = float(rng.integers(0, 8)) / 8 + 1 / 16
        idx, W = orc.resample_indices(wp, wb, U)
        q = [orc.fixed40(v) for v in np.concatenate([wp, wb])]
        F = np.cumsum(q).tolist()
        for j, i in enumerate(idx):
            u = (j + Fraction(U)) * W / nu
            lo = F[i - 1] if i > 0 else 0
            assert lo <= u < F[i], (trial, j, i)


# ---------------------------------------------------------------------------------------
# initial state (the paper leaves it open; reading: particles spread uniformly over the grid,
# velocity from the birth pdf, weight 0, so that the first cycle is all birth)
# ---------------------------------------------------------------------------------------

def test_init_state_distribution(orc):
    """Positions uniform over [0, nx r) x [0, ny r) (a wide, flat grid so that the two extents
    differ), velocity components N(0, sigma_B^2) and independent, weights exactly 0: each
    checked against its distribution within 5 standard errors."""
    p = params(orc, nx=90, ny=20, nu=60000, sigma_birth_vel=4.0, sigma_vel=0.5, seed=11)
    n = p.n_pers
    st = orc.init_state(p, n)
    r = float(np.float32(p.cell_size))
    ext = {"x": p.nx * r, "y": p.ny * r}
    for c in ("x", "y"):
        v = st[c] / ext[c]  # U(0, 1)
        assert np.all((v > 0) & (v < 1)), c
        assert abs(v.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n), c
        assert abs(v.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / n), c
        hist = np.bincount(np.minimum((v * 10).astype(int), 9), minlength=10)
        assert np.all(np.abs(hist - n / 10) < 5 * math.sqrt(n * 0.09)), c  # flat in deciles
    sB = float(np.float32(p.sigma_birth_vel))
    for c in ("vx", "vy"):
        z = st[c] / sB
        assert abs(z.mean()) < 5 / math.sqrt(n), c
        assert abs(z.var() - 1) < 5 * math.sqrt(2 / n), c
        assert abs(np.mean(z ** 4) - 3) < 5 * math.sqrt(96 / n), c  # Gaussian kurtosis
    corr = lambda a, b: np.corrcoef(a, b)[0, 1]  # noqa: E731
    for a, b in (("vx", "vy"), ("x", "y"), ("x", "vx"), ("y", "vy")):
        assert abs(corr(st[a], st[b])) < 5 / math.sqrt(n), (a, b)
    assert np.all(st["w"] == 0.0)
    # another seed or grid gives another state
    q = params(orc, nx=90, ny=20, nu=1000, seed=12)
    assert not np.array_equal(orc.init_state(q, 1000)["x"], st["x"][:1000])


# ---------------------------------------------------------------------------------------
# the exact fixed-point sums of the integer decisions against plain FP64 scans
# ---------------------------------------------------------------------------------------

def _c512_weights(orc, cycles=3):
    """Persistent (sorted) and new-born weights and rho_b of the oracle's third cycle of the
    512x512 / 2^21 + 2^18 workload."""
    wl = scenes.WORKLOADS["c512"]
    f = scenes.FILTER
    p = orc.Params(wl["nx"], wl["ny"], wl["cell"], f["dt"], f["p_s"], f["p_b"], f["sigma_pos"],
                   f["sigma_vel"], f["sigma_birth_vel"], f["alpha_free"], wl["n_pers"],
                   wl["n_born"], seed=0, grid_id=0)
    st = orc.init_state(p, p.n_pers)
    m_F = np.zeros(p.C)
    info = None
    for k, m in enumerate(scenes.measurement_sequence(wl, cycles), start=1):
        meas = {kk: np.asarray(v, np.float64) for kk, v in m.items()}
        st, m_F, info = orc.cycle(p, k, st, m_F, meas)
    return p, info


def test_fixed_point_sums_against_plain_fp64_scans(orc):
    """The integer decisions use sums of masses rounded to multiples of 2^-40 (exact in 64-bit
    integers).  On the 512x512 workload's weights, a plain sequential FP64 scan (the textbook
    CDF of Alg. 7 and the normalised born-mass scan of Alg. 5) picks the same resampling index
    and the same slot offset except where the draw or the scaled prefix lies within the
    difference of the two scans of a boundary; the counts are printed."""
    p, info = _c512_weights(orc)
    nu = p.n_pers
    wj = np.concatenate([info["sorted"]["w"], info["born"]["w"]])
    # resampling: fixed-point CDF (the oracle) vs a sequential FP64 CDF
    U = orc.resample_offset(p, 3)
    idx_fix, W_fix = orc.resample_indices(info["sorted"]["w"], info["born"]["w"], U)
    F64 = np.cumsum(wj)  # sequential FP64 sums
    W64 = F64[-1]
    u64 = (np.arange(nu) + U) * (W64 / nu)
    idx64 = np.minimum(np.searchsorted(F64, u64, side="right"), len(wj) - 1)
    q = np.floor(wj * 2.0 ** 40 + 0.5)
    Ffix = np.cumsum(q) * 2.0 ** -40  # exact integers times a power of two (below 2^53)
    eps = float(np.max(np.abs(Ffix - F64))) + abs(W_fix * 2.0 ** -40 - W64) + 4 * W64 * 2.0 ** -52
    diff = np.nonzero(idx_fix != idx64)[0]
    for j in diff:
        lo, hi = sorted((int(idx_fix[j]), int(idx64[j])))
        gap = np.min(np.abs(F64[lo:hi] - u64[j]))  # boundaries between the two choices
        assert gap <= eps, (j, gap, eps)
    print(f"resampling: {len(diff)} of {nu} indices differ (CDF difference {eps:.2e} of "
          f"W = {W64:.1f})")
    # new-born slots: fixed-point prefix vs a sequential FP64 exclusive scan of rho_b
    rho_b = info["rho_b"]
    off_fix = info["born_off"]
    E64 = np.concatenate([[0.0], np.cumsum(rho_b)])
    S64 = E64[-1]
    t64 = p.n_born * E64[:-1] / S64
    off64 = np.minimum(np.floor(t64), p.n_born).astype(np.int64)
    off64[E64[:-1] >= S64] = p.n_born
    qb = np.floor(rho_b * 2.0 ** 40 + 0.5)
    Efix = np.concatenate([[0.0], np.cumsum(qb)]) * 2.0 ** -40
    eps_b = p.n_born * (float(np.max(np.abs(Efix - E64))) / S64 + 4 * 2.0 ** -52)
    dc = np.nonzero(off_fix[:-1].astype(np.int64) != off64)[0]
    for c in dc:
        assert abs(t64[c] - round(t64[c])) <= eps_b, (c, t64[c], eps_b)
    print(f"new-born slots: {len(dc)} of {p.C} offsets differ (band {eps_b:.2e} slots)")

