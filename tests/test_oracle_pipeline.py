"""Pins of the oracle's keypoint back-map (level -> view -> source -> original image), the part
of the composed pipeline not covered by the stage modules' own pins."""
import numpy as np

from oracle import pipeline as PL
from oracle import plan as OP


def _feat(x, y, level):
    return {"x": np.asarray(x, np.int64), "y": np.asarray(y, np.int64), "level": np.asarray(level, np.int64)}


def test_identity_view_level0_maps_to_itself():
    v = OP.plan_view(200, 150, 1.0, 0.0, 0.0, 1.0)
    g = np.random.default_rng(1)
    x, y = g.integers(0, 200, 50), g.integers(0, 150, 50)
    xs, ys = PL.keypoints_to_source(_feat(x, y, np.zeros(50)), v, PL.OrbOptions(n_levels=3))
    assert np.array_equal(xs, x) and np.array_equal(ys, y)


def test_level_pixel_centres_cover_the_view_symmetrically():
    # the first and last pixel centres of level l sit half a level pixel inside [-1/2, W0 - 1/2]
    v = OP.plan_view(200, 150, 1.0, 0.0, 0.0, 1.0)
    opts = PL.OrbOptions(n_levels=4)
    dims = OP.level_dims(200, 150, 4)
    for lvl in range(4):
        wl, hl = dims[lvl]
        xs, ys = PL.keypoints_to_source(_feat([0, wl - 1], [0, hl - 1], [lvl, lvl]), v, opts)
        hx, hy = 0.5 * 200 / wl, 0.5 * 150 / hl
        assert np.allclose(xs, [hx - 0.5, 200 - hx - 0.5], atol=1e-12)
        assert np.allclose(ys, [hy - 0.5, 150 - hy - 0.5], atol=1e-12)


def test_back_map_inverts_the_view_map():
    # a tilted, rotated, scaled view: the source point of a level-0 keypoint maps forward onto it
    v = OP.plan_view(300, 220, 2.5, 0.9, 0.4, 1.3)
    g = np.random.default_rng(2)
    x, y = g.integers(0, v.width, 40), g.integers(0, v.height, 40)
    xs, ys = PL.keypoints_to_source(_feat(x, y, np.zeros(40)), v, PL.OrbOptions(n_levels=2))
    F = np.asarray(v.fwd, np.float64)
    qx = F[0, 0] * xs + F[0, 1] * ys + F[0, 2]
    qy = F[1, 0] * xs + F[1, 1] * ys + F[1, 2]
    assert np.abs(qx - x).max() < 1e-9 and np.abs(qy - y).max() < 1e-9


def test_scale_stage_factor():
    # a keypoint of a half-size source at u maps to the original at (u + 1/2) / (1/2) - 1/2 = 2u + 1/2
    v = OP.plan_view(100, 80, 1.0, 0.0, 0.0, 1.0)
    x, y = np.array([0, 10, 99]), np.array([0, 5, 79])
    xs, ys = PL.keypoints_to_source(_feat(x, y, np.zeros(3)), v, PL.OrbOptions(n_levels=1), src_scale=0.5)
    assert np.array_equal(xs, 2 * x + 0.5) and np.array_equal(ys, 2 * y + 0.5)
