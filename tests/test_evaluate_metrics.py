"""Metrics of the filter-quality evaluation, pinned to independent definitions: the mixture
variance against samples drawn from the mixture, the Mahalanobis distance against a linear
solve, the ROC area against the pairwise (Mann-Whitney) probability."""
import numpy as np
import pytest

from paper_1605_02406_amd import evaluate as ev


def test_cluster_mean_and_mixture_variance_match_samples_of_the_mixture():
    rng = np.random.default_rng(3)
    means = rng.normal(5.0, 2.0, 7)
    vars_ = rng.uniform(0.1, 3.0, 7)
    n = 400_000
    comp = rng.integers(0, 7, n)  # equal weights
    x = rng.normal(means[comp], np.sqrt(vars_[comp]))
    assert ev.cluster_mean(means) == pytest.approx(np.mean(means))
    assert ev.cluster_variance(means, vars_) == pytest.approx(np.var(x), rel=0.01)


def test_single_cell_cluster_keeps_its_variance():
    assert ev.cluster_variance(np.array([2.5]), np.array([0.7])) == pytest.approx(0.7)


def test_nees():
    assert ev.nees(3.0, 4.0, 3.0) == 0.0
    assert ev.nees(5.0, 4.0, 3.0) == pytest.approx(1.0)
    # a Gaussian estimate with the stated variance gives chi^2(1): 95 % below the level
    rng = np.random.default_rng(5)
    e = np.array([ev.nees(t, 2.0, 0.0) for t in rng.normal(0.0, np.sqrt(2.0), 20000)])
    assert np.mean(e > ev.CHI2_1_95) == pytest.approx(0.05, abs=0.006)


def test_mahalanobis_matches_a_linear_solve_and_is_rotation_invariant():
    rng = np.random.default_rng(7)
    for _ in range(50):
        A = rng.normal(size=(2, 2))
        P = A @ A.T + 0.1 * np.eye(2)
        v = rng.normal(size=2) * 3
        ref = v @ np.linalg.solve(P + 1e-6 * np.eye(2), v)
        got = ev.mahalanobis(v[0], v[1], P[0, 0], P[1, 1], P[0, 1])
        assert float(got) == pytest.approx(ref, rel=1e-9)
        th = rng.uniform(0, 2 * np.pi)
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        Pr, vr = R @ P @ R.T, R @ v
        rot = ev.mahalanobis(vr[0], vr[1], Pr[0, 0], Pr[1, 1], Pr[0, 1])
        assert float(rot) == pytest.approx(float(got), rel=1e-6)
    assert float(ev.mahalanobis(2.0, 0.0, 4.0, 1.0, 0.0, reg=0.0)) == pytest.approx(1.0)
    assert np.isinf(ev.mahalanobis(1.0, 1.0, 1.0, 1.0, 1.0, reg=0.0))  # singular P


def test_roc_area_is_the_pairwise_probability():
    rng = np.random.default_rng(11)
    pos = rng.normal(1.0, 1.0, 300).round(1)  # rounding makes ties
    neg = rng.normal(0.0, 1.0, 400).round(1)
    score = np.r_[pos, neg]
    lab = np.r_[np.ones(300, bool), np.zeros(400, bool)]
    fpr, tpr = ev.roc(score, lab)
    assert fpr[0] == tpr[0] == 0.0 and fpr[-1] == tpr[-1] == 1.0
    assert np.all(np.diff(fpr) >= 0) and np.all(np.diff(tpr) >= 0)
    pairs = (pos[:, None] > neg[None, :]).mean() + 0.5 * (pos[:, None] == neg[None, :]).mean()
    assert ev.auc(fpr, tpr) == pytest.approx(pairs, abs=1e-12)


def test_roc_extremes_and_operating_point():
    lab = np.array([1, 1, 1, 0, 0, 0, 0], bool)
    fpr, tpr = ev.roc(np.array([9, 8, 7, 3, 2, 1, 0.0]), lab)
    assert ev.auc(fpr, tpr) == pytest.approx(1.0)
    assert ev.tpr_at_fpr(fpr, tpr, 0.0) == 1.0
    fpr, tpr = ev.roc(np.array([0, 1, 2, 3, 7, 8, 9.0]), lab)
    assert ev.auc(fpr, tpr) == pytest.approx(0.0)
    assert ev.tpr_at_fpr(fpr, tpr, 0.5) == 0.0
    with pytest.raises(ValueError):
        ev.roc(np.array([1.0, 2.0]), np.array([True, True]))


def test_lanes_scene_has_static_and_moving_objects():
    sc = ev.lanes_scene()
    moving = [b for b in sc.boxes if b.vx != 0.0]
    assert len(moving) == 3 and len(sc.boxes) - len(moving) >= 8
    assert all(b.vy == 0.0 for b in sc.boxes)
    occ = sc.truth()
    assert not occ[sc.ny // 2, sc.nx // 2]  # the sensor cell is free
