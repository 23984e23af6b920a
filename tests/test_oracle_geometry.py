"""Pins of the RANSAC oracle: exact interpolation of the 4 correspondences, recovery of a
known homography, degenerate samples, outlier rejection on data with a known homography,
and the quotient of eq. (7)."""
import numpy as np

import synth
from oracle import geometry as G


def _H():
    return np.array([[0.9, 0.2, 15.0], [-0.1, 1.1, -7.0], [2e-4, -1e-4, 1.0]])


def _apply(H, p):
    q = np.c_[p, np.ones(len(p))] @ H.T
    return q[:, :2] / q[:, 2:]


def test_four_point_solution_interpolates_and_recovers():
    g = synth.rng(1)
    src = g.uniform(0, 500, (4, 2))
    dst = g.uniform(0, 500, (4, 2))
    H = G.homography_from_4(src, dst)
    assert np.abs(_apply(H, src) - dst).max() < 1e-8
    Ht = _H()
    p = g.uniform(0, 600, (4, 2))
    H2 = G.homography_from_4(p, _apply(Ht, p))
    assert np.abs(H2 - Ht).max() < 1e-9


def test_degenerate_samples():
    line = np.array([[0.0, 0.0], [10.0, 10.0], [20.0, 20.0], [5.0, 80.0]])
    ok = np.array([[0.0, 0.0], [100.0, 0.0], [0.0, 100.0], [100.0, 100.0]])
    assert G.degenerate(line) and not G.degenerate(ok)
    assert G.homography_from_4(line, ok) is None and G.homography_from_4(ok, line) is None
    scores, best, H, inl = G.ransac(line, ok, [[0, 1, 2, 3]], 2.0)
    assert scores.tolist() == [-1] and best == -1 and H is None and not inl.any()


def test_ransac_finds_the_true_inliers():
    g = synth.rng(2)
    n, n_out = 300, 90
    pa = g.uniform(0, 800, (n, 2))
    pb = _apply(_H(), pa) + g.normal(0, 0.3, (n, 2))
    bad = g.choice(n, n_out, replace=False)
    pb[bad] = g.uniform(0, 800, (n_out, 2))                   # gross outliers
    truth = np.ones(n, bool)
    truth[bad] = False
    # samples drawn among true inliers find a near-true H; the best one explains all inliers
    samples = np.stack([g.choice(n, 4, replace=False) for _ in range(400)])
    scores, best, H, inl = G.ransac(pa, pb, samples, 3.0)
    assert best >= 0 and scores[best] == scores.max()
    assert np.array_equal(inl, truth) or (inl[truth].all() and inl.sum() <= truth.sum() + 2)
    assert abs(G.inlier_ratio(int(inl.sum()), n) - (n - n_out) / n) < 0.01
    # ties go to the lowest index
    dup = np.vstack([samples[best], samples[best]])
    s2, b2, _, _ = G.ransac(pa, pb, dup, 3.0)
    assert b2 == 0 and s2[0] == s2[1]


def test_points_behind_the_camera_are_outliers():
    H = np.array([[1.0, 0, 0], [0, 1.0, 0], [-0.01, 0, 1.0]])      # w = 1 - x / 100
    pa = np.array([[50.0, 10.0], [150.0, 10.0]])
    pb = _apply(H, pa)
    r = G.residuals(H, pa, pb)
    assert r[0] < 1e-9 and np.isinf(r[1])


def test_eq7_quotient():
    assert G.inlier_ratio(45, 60) == 0.75 and G.inlier_ratio(0, 0) == 0.0


def test_refit_is_exact_on_exact_data_and_beats_the_sample():
    g = synth.rng(5)
    pa = g.uniform(0, 800, (60, 2))
    assert np.abs(G.refit_homography(pa, _apply(_H(), pa)) - _H()).max() < 1e-9
    assert G.refit_homography(pa[:3], pa[:3]) is None
    pb = _apply(_H(), pa) + g.normal(0, 0.5, (60, 2))
    H4 = G.homography_from_4(pa[:4], pb[:4])
    Hr = G.refit_homography(pa, pb)
    probe = g.uniform(0, 800, (200, 2))
    e4 = np.abs(_apply(H4, probe) - _apply(_H(), probe)).max()
    er = np.abs(_apply(Hr, probe) - _apply(_H(), probe)).max()
    assert er < e4 and er < 0.5


def test_scaling_coefficient_closed_forms():
    g = synth.rng(9)
    pa = g.uniform(0, 500, (50, 2))
    des = g.integers(0, 100, 50)
    # image B = image A scaled by 1/2 about the origin: every segment halves
    pb = pa / 2
    la = np.sqrt(((pa[1:] - pa[:-1]) ** 2).sum(axis=1))
    w = 1 - (des[:-1] + des[1:]) / 1000
    assert abs(G.scaling_coefficient(pa, pb, des) - np.sum(la / 2 * w)) < 1e-9
    assert G.scaling_coefficient(pa, pb, des) > 0 > G.scaling_coefficient(pb, pa, des)
    # a rigid motion keeps every length: f = 0
    R = np.array([[0.6, -0.8], [0.8, 0.6]])
    assert abs(G.scaling_coefficient(pa, pa @ R.T + 7.0, des)) < 1e-9
    assert G.scaling_coefficient(pa[:1], pb[:1], des[:1]) == 0.0
