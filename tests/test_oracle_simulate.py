"""Pins of the oracle's view simulation: the anti-alias blur and the Lanczos-4 warp (eqs. (3)-(4))."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import plan as P
from oracle import simulate as S


def test_lanczos_kernel_closed_forms():
    assert S.lanczos4(0.0) == 1.0
    for k in [1, 2, 3, -1, -2, -3]:
        assert abs(S.lanczos4(float(k))) < 1e-15
    for x in [4.0, -4.0, 4.5, 7.0]:
        assert S.lanczos4(x) == 0.0
    xs = np.linspace(-3.9, 3.9, 79)
    assert np.array_equal(S.lanczos4(xs), S.lanczos4(-xs))
    # a value written out from math.sin: sinc(1/2) sinc(1/8)
    v = (math.sin(math.pi / 2) / (math.pi / 2)) * (math.sin(math.pi / 8) / (math.pi / 8))
    assert S.lanczos4(0.5) == pytest.approx(v, rel=1e-14)
    # continuous at the window edge
    assert abs(S.lanczos4(4.0 - 1e-7)) < 1e-7


def _img(seed, h=40, w=48):
    g = np.random.default_rng(seed)
    return g.integers(0, 256, (h, w)).astype(np.uint8)


def test_identity_view_reproduces_input():
    A = _img(1)
    v = P.plan_view(A.shape[1], A.shape[0], 1.0, 0.0)
    V, mask, U = S.simulate_view(A, v)
    assert mask.all()
    assert np.array_equal(U, A)
    assert np.abs(V - A).max() < 1e-9


def test_quarter_turn_is_exact_rotation():
    A = _img(2)
    v = P.plan_view(A.shape[1], A.shape[0], 1.0, math.pi / 2)
    V, mask, U = S.simulate_view(A, v)
    assert mask.all()
    assert np.array_equal(U, np.rot90(A, -1))


def test_half_turn_is_exact_rotation():
    A = _img(3)
    v = P.plan_view(A.shape[1], A.shape[0], 1.0, 0.0, psi=math.pi)
    V, mask, U = S.simulate_view(A, v)
    assert mask.all()
    assert np.array_equal(U, A[::-1, ::-1])


@pytest.mark.parametrize("t,phi", [(2.0, 0.5), (4.0, 2.0), (math.sqrt(2), 1.2)])
def test_constant_stays_constant(t, phi):
    A = np.full((50, 60), 77, np.uint8)
    v = P.plan_view(60, 50, t, phi, psi=0.3)
    V, mask, U = S.simulate_view(A, v)
    assert np.abs(V[mask] - 77).max() < 1e-9
    assert np.all(U[mask] == 77) and np.all(U[~mask] == 0)


def test_warp_reproduces_band_limited_image():
    H, W = 80, 90
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)

    def f(x, y):
        return 128 + 60 * np.sin(2 * np.pi * (0.03 * x + 0.02 * y)) + 40 * np.cos(2 * np.pi * (0.05 * x - 0.04 * y))

    src = f(xx, yy)
    v = P.plan_view(W, H, 1.7, 0.7, psi=-0.4, s=1.3)
    V, mask = S.warp_lanczos4(src, v)
    px, py = S.view_coords(v)
    inner = mask & (px > 5) & (px < W - 6) & (py > 5) & (py < H - 6)
    assert inner.sum() > 1000
    # normalised Lanczos-4 reproduces low frequencies to ~0.35 % of their amplitude (100 here);
    # a wrong tap sign or a transposed map would be off by tens of gray levels
    assert np.abs(V[inner] - f(px[inner], py[inner])).max() < 0.6


def test_warp_matches_scalar_brute_force():
    A = _img(4, 24, 24).astype(np.float64)
    v = P.plan_view(24, 24, 1.9, 0.8, psi=0.25, s=1.1)
    V, mask = S.warp_lanczos4(A, v)

    def L(x):
        if x == 0:
            return 1.0
        if abs(x) >= 4:
            return 0.0
        return (math.sin(math.pi * x) / (math.pi * x)) * (math.sin(math.pi * x / 4) / (math.pi * x / 4))

    G = v.inv
    for qy in range(v.height):
        for qx in range(v.width):
            px = G[0, 0] * qx + G[0, 1] * qy + G[0, 2]
            py = G[1, 0] * qx + G[1, 1] * qy + G[1, 2]
            inside = -0.5 <= px <= 23.5 and -0.5 <= py <= 23.5
            assert inside == mask[qy, qx]
            if not inside:
                assert V[qy, qx] == 0.0
                continue
            x0, y0 = math.floor(px), math.floor(py)
            num = sx = sy = 0.0
            for j in range(-3, 5):
                wy = L(j - (py - y0))
                sy += wy
                for i in range(-3, 5):
                    wx = L(i - (px - x0))
                    num += wx * wy * A[min(max(y0 + j, 0), 23), min(max(x0 + i, 0), 23)]
            for i in range(-3, 5):
                sx += L(i - (px - x0))
            assert V[qy, qx] == pytest.approx(num / (sx * sy), abs=1e-9)


def test_blur_axis_aligned_equals_convolve1d():
    A = _img(5, 45, 52)
    for phi, axis in [(0.0, 1), (math.pi / 2, 0)]:
        sigma = 0.8 * math.sqrt(4 - 1)
        u = (math.cos(phi), -math.sin(phi))
        major, m, k, g = S.blur_taps(sigma, u)
        assert abs(m) < 1e-15
        assert g.sum() == pytest.approx(1.0, abs=1e-15)
        got = S.directional_blur(A, sigma, u)
        ref = ndi.convolve1d(A.astype(np.float64), g, axis=axis, mode="nearest")
        assert np.abs(got - ref).max() < 1e-10


@pytest.mark.parametrize("phi", [0.3, 0.9, 1.9, 2.7])
def test_blur_preserves_ramps_and_constants(phi):
    H, W = 70, 80
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    ramp = 3.0 * xx - 2.0 * yy + 10.0
    u = (math.cos(phi), -math.sin(phi))
    sigma = 0.8 * math.sqrt(8 - 1)
    out = S.directional_blur(ramp, sigma, u)
    K = S.blur_taps(sigma, u)[2].max() + 2
    inner = (slice(K, H - K), slice(K, W - K))
    assert np.abs(out[inner] - ramp[inner]).max() < 1e-9
    const = S.directional_blur(np.full((H, W), 42.0), sigma, u)
    assert np.abs(const - 42.0).max() < 1e-12


@pytest.mark.parametrize("phi", [0.25, 0.8, 1.4, 2.3])
def test_blur_impulse_response_is_along_u(phi):
    n = 121
    A = np.zeros((n, n))
    A[60, 60] = 1.0
    sigma = 0.8 * math.sqrt(16 - 1)
    u = np.array([math.cos(phi), -math.sin(phi)])
    out = S.directional_blur(A, sigma, u)
    # the response of a line filter at an impulse is the filter mirrored: its mass lies along u
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    w = out / out.sum()
    dx, dy = xx - 60, yy - 60
    cov = np.array([[(w * dx * dx).sum(), (w * dx * dy).sum()], [(w * dx * dy).sum(), (w * dy * dy).sum()]])
    perp = np.array([-u[1], u[0]])
    along = u @ cov @ u
    across = perp @ cov @ perp
    assert along == pytest.approx(sigma * sigma, rel=0.12)
    assert across < 0.3


def test_quantize_rounds_half_to_even_and_clamps():
    got = S.quantize(np.array([0.5, 1.5, 2.5, -3.0, 300.0, 254.5, 7.49]))
    assert got.tolist() == [0, 2, 2, 0, 255, 254, 7]


# ---------------------------------------------------------------------------- scale stage

def test_scale_identity_and_constant():
    A = _img(11, 30, 41)
    V, U = S.scale_image(A, 1.0)
    assert np.array_equal(U, A)
    for s in (0.5, 0.25, 0.8, 1.5):
        V, U = S.scale_image(np.full((40, 52), 61, np.uint8), s)
        assert np.abs(V - 61).max() < 1e-9 and U.shape == P.scaled_size(52, 40, s)[::-1]


def test_scale_half_on_block_constant_image():
    """s = 1/2 of an image that is constant on 2x2 blocks: output pixel q samples the source
    at 2q + 1/2, between the two pixels of its block; interior values reproduce the blocks up
    to the anti-alias blur, which is exact on constants."""
    rng = np.random.default_rng(12)
    blocks = rng.integers(60, 200, (12, 14)).astype(np.float64)
    A = np.kron(blocks, np.ones((2, 2))).astype(np.uint8)
    # smooth variation only: the blur and the interpolation reproduce a linear ramp exactly
    yy, xx = np.mgrid[0:24, 0:28].astype(np.float64)
    ramp = 2.0 * xx + 3.0 * yy + 10.0
    V, U = S.scale_image(ramp.astype(np.uint8), 0.5)
    qy, qx = np.mgrid[0:12, 0:14].astype(np.float64)
    exp = 2.0 * (2 * qx + 0.5) + 3.0 * (2 * qy + 0.5) + 10.0
    inner = (slice(4, 8), slice(4, 10))
    assert np.abs(V[inner] - exp[inner]).max() < 0.35     # Lanczos-4 ripple on a ramp + blur rounding
    assert V.shape == (12, 14)


def test_scale_maps_points_consistently():
    """A bright square moves to the scaled position: centroid of the scaled image = (c + 1/2) s - 1/2."""
    A = np.zeros((80, 80), np.uint8)
    A[30:40, 44:54] = 200
    for s in (0.5, 0.25, 2.0):
        V, U = S.scale_image(A, s)
        yy, xx = np.mgrid[0:V.shape[0], 0:V.shape[1]].astype(np.float64)
        w = np.clip(V, 0, None)
        cx, cy = (w * xx).sum() / w.sum(), (w * yy).sum() / w.sum()
        assert abs(cx - ((48.5 + 0.5) * s - 0.5)) < 0.05 * max(1, s) + 0.02
        assert abs(cy - ((34.5 + 0.5) * s - 0.5)) < 0.05 * max(1, s) + 0.02


def test_sigma_follows_net_compression():
    v = P.plan_view(64, 64, 4.0, 0.3, s=2.0)
    assert v.sigma == pytest.approx(0.8 * math.sqrt(3.0))
    assert P.plan_view(64, 64, 2.0, 0.3, s=2.0).sigma == 0.0
    assert P.plan_view(64, 64, 1.0, 0.0, s=3.0).sigma == 0.0


def test_nearest_identity_shift_and_ties():
    img = np.random.default_rng(4).integers(0, 256, (30, 41)).astype(np.uint8)
    v = P.plan_view(41, 30, 1.0, 0.0)
    V, M, U = S.simulate_view(img, v, "nearest")
    assert M.all() and np.array_equal(U, img)
    # half-pixel positions take the pixel above/right (floor(p + 1/2))
    px = np.array([0.5, 1.5, 2.49999, 2.5, -0.5, 40.5])
    py = np.array([0.5, 0.0, 0.0, 0.0, -0.5, 29.5])
    got = S.nearest_sample(img, px, py)
    assert np.array_equal(got, [img[1, 1], img[0, 2], img[0, 2], img[0, 3], img[0, 0], img[29, 40]])


def test_nearest_quarter_turn_is_rot90():
    img = np.random.default_rng(5).integers(0, 256, (24, 24)).astype(np.uint8)
    for k, phi in ((1, math.pi / 2), (2, math.pi), (3, 3 * math.pi / 2)):
        v = P.plan_view(24, 24, 1.0, phi)
        _, M, U = S.simulate_view(img, v, "nearest")
        assert M.all()
        assert any(np.array_equal(U, np.rot90(img, kk)) for kk in (k, -k))


def test_nearest_brute_force_on_a_tilted_view():
    img = np.random.default_rng(6).integers(0, 256, (20, 26)).astype(np.uint8)
    v = P.plan_view(26, 20, 2.0, 0.4, 0.3, 1.3)
    B = S.directional_blur(img, v.sigma, v.u)
    V, M = S.warp_nearest(B, v)
    G = v.inv
    for qy in range(v.height):
        for qx in range(v.width):
            px = G[0, 0] * qx + G[0, 1] * qy + G[0, 2]
            py = G[1, 0] * qx + G[1, 1] * qy + G[1, 2]
            inside = -0.5 <= px <= 25.5 and -0.5 <= py <= 19.5
            assert M[qy, qx] == inside
            if inside:
                ix = min(max(int(math.floor(px + 0.5)), 0), 25)
                iy = min(max(int(math.floor(py + 0.5)), 0), 19)
                assert V[qy, qx] == B[iy, ix]
