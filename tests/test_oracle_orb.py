"""Pins of the oracle's ORB steps (pyramid, FAST-9, Harris, orientation, smoothing, rBRIEF)."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

import synth
from oracle import orb as O


def _img(seed, h, w):
    return np.random.default_rng(seed).integers(0, 256, (h, w)).astype(np.uint8)


# ---------------------------------------------------------------------------- pyramid

@pytest.mark.parametrize("n_src,n_dst", [(1024, 853), (768, 640), (100, 83), (45, 38), (7, 6), (1, 1)])
def test_resample_index_matches_real_definition(n_src, n_dst):
    i0, i1, w0, w1 = O._resample_index(n_dst, n_src)
    for d in range(n_dst):
        src = (d + 0.5) * n_src / n_dst - 0.5
        q = math.floor(src * 2048 + 0.5)
        a, b = q >> 11, q & 2047
        if a >= n_src - 1:
            a, b = n_src - 1, 0
        assert (i0[d], w1[d], w0[d]) == (a, b, 2048 - b)
        assert i1[d] == min(a + 1, n_src - 1)


def test_pyramid_constant_and_ramp():
    P = np.full((60, 70), 93, np.uint8)
    out, m = O.pyr_down(P, np.ones_like(P, bool), 58, 50)
    assert np.all(out == 93) and m.all()
    # a horizontal ramp is reproduced at the mapped position to within rounding
    ramp = np.tile(np.arange(200, dtype=np.uint8), (10, 1))
    out, _ = O.pyr_down(ramp, np.ones(ramp.shape, bool), 167, 8)
    x = (np.arange(167) + 0.5) * 200 / 167 - 0.5
    assert np.abs(out[3].astype(float) - np.clip(x, 0, 199)).max() <= 0.5 + 1 / 2048 * 200


def test_pyramid_mask_is_and_of_footprint():
    P = _img(1, 30, 30)
    M = np.ones((30, 30), bool)
    M[10, 17] = False
    out, m = O.pyr_down(P, M, 25, 25)
    i0, i1, _, _ = O._resample_index(25, 30)
    for y in range(25):
        for x in range(25):
            exp = all(M[yy, xx] for yy in (i0[y], i1[y]) for xx in (i0[x], i1[x]))
            assert m[y, x] == exp


# ---------------------------------------------------------------------------- FAST

def _segment_test(I, x, y, T):
    """Literal FAST-9 segment test: 9 contiguous circle pixels all brighter than I_p + T
    or all darker than I_p - T."""
    p = int(I[y, x])
    ring = [int(I[y + dy, x + dx]) for dx, dy in O.CIRCLE]
    for s in range(16):
        arc = [ring[(s + j) % 16] for j in range(9)]
        if all(c > p + T for c in arc) or all(c < p - T for c in arc):
            return True
    return False


def test_fast_score_is_the_segment_test_threshold():
    I = _img(2, 18, 20)
    # smooth-ish structure so that some pixels are corners at moderate thresholds
    I = (ndi.uniform_filter(I.astype(float), 2) * 1.0).astype(np.uint8)
    V = O.fast_score(I)
    for y in range(3, 15):
        for x in range(3, 17):
            for T in (0, 5, 20, 60):
                assert (V[y, x] > T) == _segment_test(I, x, y, T)


def test_fast_constant_image_has_no_corners():
    I = np.full((60, 60), 100, np.uint8)
    assert (O.fast_score(I)[3:-3, 3:-3] <= 0).all()
    xs, ys = O.fast_candidates(I, np.ones_like(I, bool), 20, 22)
    assert xs.size == 0


def test_fast_isolated_bright_pixel():
    I = np.full((50, 50), 40, np.uint8)
    I[25, 25] = 140
    V = O.fast_score(I)
    assert V[25, 25] == 100
    xs, ys = O.fast_candidates(I, np.ones_like(I, bool), 20, 22)
    assert list(zip(xs, ys)) == [(25, 25)]


def test_fast_score_rotates_with_the_image():
    I = _img(3, 40, 40)
    V = O.fast_score(I)
    Vr = O.fast_score(np.rot90(I))
    assert np.array_equal(np.rot90(V), Vr)


def test_fast_nms_brute_force():
    g = np.random.default_rng(4)
    I = ndi.gaussian_filter(g.integers(0, 256, (90, 90)).astype(float), 1.0)
    I = np.clip((I - I.mean()) * 6 + 128, 0, 255).astype(np.uint8)
    M = np.ones(I.shape, bool)
    M[:, 80:] = False
    T, B = 10, 22
    xs, ys = O.fast_candidates(I, M, T, B)
    V = O.fast_score(I)
    got = set(zip(xs.tolist(), ys.tolist()))
    exp = set()
    W = I.shape[1]
    for y in range(B, 90 - B):
        for x in range(B, 90 - B):
            if not V[y, x] > T:
                continue
            ok = True
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dx, dy) == (0, 0) or not V[y + dy, x + dx] > T:
                        continue
                    rq, rp = (y + dy) * W + x + dx, y * W + x
                    if V[y + dy, x + dx] > V[y, x] or (V[y + dy, x + dx] == V[y, x] and rq < rp):
                        ok = False
            if ok and all(M[y + a, x + b] for a in (-B, B) for b in (-B, B)):
                exp.add((x, y))
    assert got == exp and len(exp) > 5
    # survivors are never 8-adjacent
    for (x, y) in got:
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                if (dx, dy) != (0, 0):
                    assert (x + dx, y + dy) not in got


# ---------------------------------------------------------------------------- Harris

def test_harris_equals_scipy_sobel_and_box_sums():
    I = _img(5, 40, 44).astype(np.int64)
    sx = ndi.sobel(I, axis=1, mode="constant")   # x derivative, int64 exact
    sy = ndi.sobel(I, axis=0, mode="constant")
    box = np.ones((7, 7), np.int64)
    a = ndi.correlate(sx * sx, box, mode="constant")
    b = ndi.correlate(sy * sy, box, mode="constant")
    c = ndi.correlate(sx * sy, box, mode="constant")
    ys, xs = np.mgrid[5:35, 5:39]
    xs, ys = xs.ravel(), ys.ravel()
    R = O.harris_response(I.astype(np.uint8), xs, ys)
    det = a[ys, xs] * b[ys, xs] - c[ys, xs] ** 2
    tr = a[ys, xs] + b[ys, xs]
    assert np.array_equal(R, 25 * det - tr * tr)
    # integer form ranks like the textbook det - 0.04 tr^2
    f = det.astype(np.float64) - 0.04 * tr.astype(np.float64) ** 2
    assert np.array_equal(np.argsort(-R, kind="stable"), np.argsort(-f * 25, kind="stable"))


def test_harris_pure_gradient_closed_form():
    I = np.tile((np.arange(40) * 5).astype(np.uint8), (40, 1))
    R = O.harris_response(I, np.array([20]), np.array([20]))
    ix = 5 * 2 * (1 + 2 + 1)            # Sobel of a slope-5 ramp
    a = 49 * ix * ix
    assert R[0] == -a * a


def test_select_top_order():
    R = np.array([5, 9, 9, 1, 9, 7])
    raster = np.array([10, 40, 30, 0, 50, 20])
    assert O.select_top(R, raster, 4).tolist() == [2, 1, 4, 5]


# ---------------------------------------------------------------------------- orientation

def test_orientation_table_first_entries():
    C, S = O.orientation_table()
    assert C[:4].tolist() == [1048576, 1025662, 957922, 848316]
    assert S[0] == 0 and C[15] == -C[0] and S[22] == -S[7]


def test_disk_has_709_pixels():
    dx, dy = O.disk_offsets()
    assert dx.size == 709


@pytest.mark.parametrize("alpha_deg", [0, 12, 47, 88, 133, 180, 181, 265, 301, 350])  # none on a half-bin tie
def test_ramp_orientation(alpha_deg):
    a = math.radians(alpha_deg)
    yy, xx = np.mgrid[0:41, 0:41].astype(np.float64)
    I = np.clip(np.rint(128 + 3.0 * ((xx - 20) * math.cos(a) + (yy - 20) * math.sin(a))), 0, 255).astype(np.uint8)
    b = O.orientation_bins(I, np.array([20]), np.array([20]))[0]
    assert b == round(alpha_deg / 12.0) % 30


def test_orientation_half_turn():
    I = _img(6, 61, 61)
    b = O.orientation_bins(I, np.array([30]), np.array([30]))[0]
    b2 = O.orientation_bins(I[::-1, ::-1], np.array([30]), np.array([30]))[0]
    assert b2 == (b + 15) % 30


# ---------------------------------------------------------------------------- smoothing + BRIEF

def test_smooth_equals_scipy_correlate():
    I = _img(7, 33, 41).astype(np.int64)
    w = O.SMOOTH_TAPS
    h = ndi.correlate1d(I, w, axis=1, mode="nearest")
    v = ndi.correlate1d(h, w, axis=0, mode="nearest")
    assert np.array_equal(O.smooth(I.astype(np.uint8)), ((v + (1 << 15)) >> 16).astype(np.uint8))
    assert np.all(O.smooth(np.full((9, 9), 200, np.uint8)) == 200)


def test_brief_constant_patch_is_zero():
    pat = synth.brief_pattern()
    Sm = np.full((60, 60), 31, np.uint8)
    d = O.brief_descriptors(Sm, [30], [30], [7], pat)
    assert not d.any()


def test_brief_bit_layout():
    # every test compares a = p + (1, 0) against b = p: bit = [S(a) < S(b)]
    pat = np.zeros((256, 4), np.int8)
    pat[:, 0] = 1
    Sm = np.zeros((10, 10), np.uint8)
    Sm[5, 6] = 9            # S(a) = 9, S(b) = 0: every bit is 0
    assert not O.brief_descriptors(Sm, [5], [5], [0], pat).any()
    pat[3] = (0, 0, 1, 0)   # test 3 swaps the points: S(p) = 0 < S(p + (1, 0)) = 9
    pat[200] = (0, 0, 1, 0)
    d = O.brief_descriptors(Sm, [5], [5], [0], pat)
    exp = np.zeros(32, np.uint8)
    exp[0] = 1 << 3
    exp[25] = 1 << 0        # test 200 -> byte 25, bit 0
    assert np.array_equal(d[0], exp)


def test_steering_is_odd_symmetric_and_bounded():
    pat = synth.brief_pattern()
    for b in range(30):
        s = O.steer_pattern(pat, b)
        s2 = O.steer_pattern(pat, (b + 15) % 30)
        assert np.array_equal(s, -s2)
        assert np.abs(s).max() <= O.BORDER - 1
    assert np.array_equal(O.steer_pattern(pat, 0), pat.astype(np.int64))


def test_extract_is_equivariant_under_half_turn():
    pat = synth.brief_pattern()
    sc = synth.make_scene(160, 140, 30, 25, seed=11)
    A = synth.render(sc, np.eye(2), np.zeros(2), 160, 140, noise_seed=3)
    M = np.ones(A.shape, bool)
    f = O.extract_view(A, M, [(160, 140)], [400], 20, pat)
    g = O.extract_view(A[::-1, ::-1].copy(), M, [(160, 140)], [400], 20, pat)
    assert len(f["x"]) > 20
    ka = {(int(x), int(y)): i for i, (x, y) in enumerate(zip(f["x"], f["y"]))}
    common = 0
    for j, (x, y) in enumerate(zip(g["x"], g["y"])):
        i = ka.get((159 - int(x), 139 - int(y)))
        if i is None:
            continue
        common += 1
        assert g["harris"][j] == f["harris"][i]
        if g["bin"][j] == (f["bin"][i] + 15) % 30:
            assert np.array_equal(g["desc"][j], f["desc"][i])
    assert common >= 0.8 * len(f["x"])


def test_extract_canonical_order():
    pat = synth.brief_pattern()
    sc = synth.make_scene(200, 180, 40, 30, seed=12)
    A = synth.render(sc, np.eye(2), np.zeros(2), 200, 180, noise_seed=5)
    dims = [(200, 180), (167, 150), (139, 125)]
    f = O.extract_view(A, np.ones(A.shape, bool), dims, [60, 40, 30], 20, pat)
    lv = f["level"]
    assert np.all(np.diff(lv) >= 0)
    for l in range(3):
        sel = lv == l
        R = f["harris"][sel]
        rs = f["y"][sel] * dims[l][0] + f["x"][sel]
        key = list(zip(-R, rs))
        assert key == sorted(key)
        assert sel.sum() <= [60, 40, 30][l]
