"""Pins of the oracle's view planning (sampling rule of Sec. III.B, camera map of eq. (2))."""
import math

import numpy as np
import pytest

from oracle import plan as P


def test_views_per_tilt_match_eq11(golden):
    grid = P.sampling_grid(5)
    ts = [t for t, _ in grid]
    counts = [sum(1 for t in ts if abs(t - P.tilt(i)) < 1e-12) for i in range(6)]
    assert counts == golden["views_per_tilt"]["value"]
    assert len(grid) == golden["views_total_n5"]["value"]


def test_tilts_are_powers_of_sqrt2(golden):
    a = golden["sampling_rule"]["a"]
    for i in range(8):
        assert P.tilt(i) == pytest.approx(a ** i, rel=1e-15)
    # even exponents are exact powers of two (the k b / t < 180 test sits on its boundary there)
    assert P.tilt(2) == 2.0 and P.tilt(4) == 4.0 and P.tilt(6) == 8.0


def test_longitudes_below_180_and_maximal():
    for i in range(8):
        t = P.tilt(i)
        phis = [math.degrees(f) for tt, f in P.sampling_grid(i) if tt == t]
        step = 72.0 / t
        assert phis[0] == 0.0
        assert all(p < 180.0 for p in phis)
        # the next longitude would reach or pass 180 deg
        assert phis[-1] + step >= 180.0 - 1e-9
        assert np.allclose(np.diff(phis), step)


def test_printed_best_parameters_lie_on_the_grid(golden):
    g = golden["best_params_graffiti_1_5_ds0"]
    grid = P.sampling_grid(5)
    # the printed longitude is a grid longitude (k = 7 at t = 2 sqrt 2, k = 14 at t = 4 sqrt 2) ...
    hits = [(t, f) for t, f in grid if abs(math.degrees(f) - g["best_phi_deg"]) < 5e-4]
    assert len(hits) == 2
    # ... and exactly one of them has the printed latitude theta = arccos(1/t) (printed rounded to 70 deg)
    near = [t for t, f in hits if abs(math.degrees(math.acos(1.0 / t)) - g["best_theta_deg"]) < 1.0]
    assert near == [2.0 * math.sqrt(2.0)]


def test_identity_view():
    v = P.plan_view(37, 21, 1.0, 0.0)
    assert (v.width, v.height) == (37, 21)
    assert np.array_equal(v.fwd, np.array([[1.0, 0, 0], [0, 1.0, 0]]))
    assert v.sigma == 0.0


def test_quarter_turn_canvas_swaps_sides():
    v = P.plan_view(37, 21, 1.0, math.pi / 2)
    assert (v.width, v.height) == (21, 37)


@pytest.mark.parametrize("t,phi,psi,s", [(2.0, 0.3, 0.0, 1.0), (4 * math.sqrt(2), 2.9, 0.7, 1.0),
                                         (math.sqrt(2), 1.1, -0.4, 0.5)])
def test_canvas_tightly_contains_mapped_source(t, phi, psi, s):
    W, H = 101, 57
    v = P.plan_view(W, H, t, phi, psi, s)
    c = np.array([[-0.5, W - 0.5, -0.5, W - 0.5], [-0.5, -0.5, H - 0.5, H - 0.5]])
    q = v.fwd[:, :2] @ c + v.fwd[:, 2:3]
    assert q.min(axis=1) == pytest.approx([-0.5, -0.5], abs=1e-9)
    assert np.all(q.max(axis=1) <= np.array([v.width, v.height]) - 0.5 + 1e-9)
    assert np.all(q.max(axis=1) > np.array([v.width, v.height]) - 1.5)
    # inverse map really inverts the forward map
    comp = v.inv[:, :2] @ v.fwd[:, :2]
    assert np.allclose(comp, np.eye(2), atol=1e-12)
    assert np.allclose(v.inv[:, :2] @ v.fwd[:, 2] + v.inv[:, 2], 0, atol=1e-9)
    # area scales by s^2 / t
    assert abs(np.linalg.det(v.fwd[:, :2])) == pytest.approx(s * s / t, rel=1e-12)


@pytest.mark.parametrize("phi", [0.0, 0.4, 1.3, math.pi / 2, 2.2, 3.0])
def test_blur_direction_is_the_compressed_direction(phi):
    t = 2.0 * math.sqrt(2)
    v = P.plan_view(64, 64, t, phi, psi=0.9)
    L = v.fwd[:, :2]
    u = np.array(v.u)
    perp = np.array([-u[1], u[0]])
    assert np.linalg.norm(L @ u) == pytest.approx(1.0 / t, rel=1e-12)
    assert np.linalg.norm(L @ perp) == pytest.approx(1.0, rel=1e-12)
    assert v.sigma == pytest.approx(0.8 * math.sqrt(t * t - 1))


def test_level_dims_and_quotas():
    dims = P.level_dims(1024, 768, 8)
    assert dims[0] == (1024, 768)
    for l, (w, h) in enumerate(dims):
        assert abs(w - 1024 / 1.2 ** l) <= 0.5 and abs(h - 768 / 1.2 ** l) <= 0.5
    for n, L in [(300, 3), (1000, 8), (500, 8), (2000, 8)]:
        q = P.level_quotas(n, L)
        assert sum(q) == n
        assert all(a >= b for a, b in zip(q, q[1:]))
        # proportional to level area: consecutive ratios near 1.44
        assert q[1] / q[2] == pytest.approx(1.44, rel=0.05)
        # exact: level l >= 1 gets floor(N r^l / sum_m r^m) with r = 1.2^-2 = 25/36, evaluated in
        # rational arithmetic; level 0 takes the rest
        from fractions import Fraction
        r = Fraction(25, 36)
        tot = sum(r ** m for m in range(L))
        upper = [int(n * r ** l // tot) for l in range(1, L)]
        assert q == [n - sum(upper)] + upper
    # the values worked out by hand for the tiny and full-size workloads (300 points over 3 levels,
    # 1000 over 8): flooring, not rounding, on the upper levels
    assert P.level_quotas(300, 3) == [139, 95, 66]
    assert P.level_quotas(1000, 8) == [325, 224, 155, 108, 75, 52, 36, 25]


def test_coupled_scale_schedule_matches_eq11():
    """s_i = 1 + i delta_s on tilt index i; view counts per tilt stay 3, 4, 5, 8, 10, 15 and the
    area factors are (1 + i delta_s)^2 as in eq. (11)."""
    g = P.sampling_grid_scaled(5, 0.5)
    assert len(g) == 45
    for i, n in enumerate((3, 4, 5, 8, 10, 15)):
        rows = [r for r in g if abs(r[0] - P.tilt(i)) < 1e-12]
        assert len(rows) == n and all(abs(r[2] - (1 + 0.5 * i)) < 1e-15 for r in rows)
    assert [r[:2] for r in P.sampling_grid_scaled(5, 0.0)] == P.sampling_grid(5)
