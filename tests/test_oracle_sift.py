"""The SIFT oracle (oracle/sift.py) pinned by closed forms, brute force and invariances."""
import math

import numpy as np
import pytest

import synth
from oracle import sift as S


def _scene(w, h, n_blobs, n_rects, seed):
    sc = synth.make_scene(w, h, n_blobs, n_rects, seed)
    return synth.render(sc, np.eye(2), np.zeros(2), w, h, noise_seed=seed, supersample=2)


def test_taps_are_the_sampled_gaussian():
    for sigma in (0.8, 1.2263, 1.52, 1.6, 3.09):
        w = S.gaussian_taps(sigma)
        r = (len(w) - 1) // 2
        assert r == math.ceil(4 * sigma)
        k = np.arange(-r, r + 1, dtype=np.float64)
        ref = np.exp(-k * k / (2 * sigma * sigma))
        ref /= ref.sum()
        assert np.array_equal(w, ref.astype(np.float32))
        assert np.array_equal(w, w[::-1])
        assert abs(float(w.astype(np.float64).sum()) - 1.0) < 1e-6
        if sigma >= 1.0:     # second moment of the sampled Gaussian, truncated at 4 sigma
            assert abs(float((k * k * w).sum()) - sigma * sigma) < 2e-3 * sigma * sigma


def test_blur_of_constant_and_of_an_impulse():
    c = np.full((37, 53), 117.0, np.float32)
    out = S.blur(c, 1.6)
    assert np.abs(out - 117.0).max() <= 117.0 * 4e-7 * 20
    imp = np.zeros((41, 41), np.float32)
    imp[20, 20] = 1.0
    w = S.gaussian_taps(2.0)
    r = (len(w) - 1) // 2
    out = S.blur(imp, 2.0)
    # every output is one rounded product of a row tap and a column tap
    ref = np.zeros_like(imp)
    ref[20 - r:21 + r, 20 - r:21 + r] = w[:, None] * w[None, :]
    assert np.array_equal(out, ref)


def test_blur_replicates_the_border():
    a = np.zeros((20, 20), np.float32)
    a[:, 0] = 100.0
    out = S.blur(a, 1.0)
    # the edge column stands for the columns beyond it: its blur keeps more than half its value
    w = S.gaussian_taps(1.0)
    r = (len(w) - 1) // 2
    assert abs(float(out[10, 0]) - 100.0 * float(w[r:].astype(np.float64).sum())) < 1e-3


def test_layer_sigmas_compose_to_the_octave_scales():
    base, inc = S.layer_sigmas()
    total = math.sqrt(S.SIGMA_IN ** 2 + base ** 2)
    assert abs(total - S.SIGMA0) < 1e-12
    for k, s in enumerate(inc, start=1):
        total = math.sqrt(total ** 2 + s ** 2)
        assert abs(total - S.SIGMA0 * 2 ** (k / S.N_LAYERS)) < 1e-12


def test_octave_count_and_sizes():
    assert S.octave_count(1024, 768) == 6
    assert S.octave_count(129, 129) == 4
    g = S.gaussian_pyramid(np.zeros((129, 129), np.uint8))
    assert [layer[0].shape for layer in g] == [(129, 129), (65, 65), (33, 33), (17, 17)]
    assert all(len(layer) == S.N_LAYERS + 3 for layer in g)
    # the next octave starts from every second pixel of G_s
    a = _scene(129, 129, 10, 8, 3)
    g = S.gaussian_pyramid(a)
    assert np.array_equal(g[1][0], g[0][S.N_LAYERS][0::2, 0::2])


def test_constant_image_has_no_candidate():
    g = S.gaussian_pyramid(np.full((64, 64), 90, np.uint8))
    d = S.dog_pyramid(g)
    # float32 blurs of a constant move it by rounding only
    assert max(float(np.abs(x).max()) for oc in d for x in oc) < 1e-3
    assert S.find_candidates(d) == []


def test_candidates_equal_a_brute_force_loop():
    a = _scene(72, 64, 25, 20, 11)
    d = S.dog_pyramid(S.gaussian_pyramid(a))
    got = S.find_candidates(d)
    pre = 0.5 * S.contrast_threshold()
    ref = []
    for o, D in enumerate(d):
        H, W = D[0].shape
        for k in range(1, S.N_LAYERS + 1):
            for y in range(S.BORDER, H - S.BORDER):
                for x in range(S.BORDER, W - S.BORDER):
                    v = float(D[k][y, x])
                    if not abs(v) > pre:
                        continue
                    nbs = [float(D[k + a_][y + b_, x + c_]) for a_ in (-1, 0, 1) for b_ in (-1, 0, 1)
                           for c_ in (-1, 0, 1) if (a_, b_, c_) != (0, 0, 0)]
                    if (v > 0 and all(v > q for q in nbs)) or (v < 0 and all(v < q for q in nbs)):
                        ref.append((o, k, y, x))
    assert got == ref and len(ref) > 5


def _quadratic_stack(x0, y0, s0, H=24, W=24, n=5):
    """D_k(y, x) = 40 - (x - x0)^2 - 2 (y - y0)^2 - 3 (k - s0)^2 + 0.5 (x - x0)(y - y0), float32
    (exact: small integers and halves)."""
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    return [(40 - (xx - x0) ** 2 - 2 * (yy - y0) ** 2 - 3 * (k - s0) ** 2 + 0.5 * (xx - x0) * (yy - y0))
            .astype(np.float32) for k in range(n)]


def test_fit_recovers_the_offset_of_a_quadratic():
    x0, y0, s0 = 11.25, 12.375, 2.125     # binary fractions: the float32 samples are exact
    D = _quadratic_stack(x0, y0, s0)
    F = S.fit(D, 2, 12, 11)
    off = np.array(F["n"]) / F["det"]
    assert np.allclose(off, [x0 - 11, y0 - 12, s0 - 2], atol=1e-12)
    # from one sample away in x and in scale, the fit steps onto the extremum and stops there
    loc = S.localise(D, 0, 1, 12, 12, contrast=0.0, edge=1e9)
    assert loc is not None and (loc["xi"], loc["yi"], loc["layer"]) == (11, 12, 2)
    assert abs(loc["x"] - x0) < 1e-12 and abs(loc["y"] - y0) < 1e-12


def test_fit_rejections():
    D = _quadratic_stack(11.25, 12.375, 2.125)
    # contrast: |D(x^)| = 40 - ... is about 40; a threshold above it rejects
    assert S.localise(D, 0, 2, 12, 11, contrast=40.5 * 3 / 255) is None
    assert S.localise(D, 0, 2, 12, 11, contrast=39.0 * 3 / 255) is not None
    # edge: principal curvatures -2 and -4 (ratio 2): tr^2 / det = 36 / 7.75 > (r + 1)^2 / r for r = 1.1
    assert S.localise(D, 0, 2, 12, 11, contrast=0.0, edge=1.1) is None
    assert S.localise(D, 0, 2, 12, 11, contrast=0.0, edge=3.0) is not None
    # a saddle in space (det of the 2x2 Hessian < 0) is rejected
    yy, xx = np.mgrid[0:24, 0:24].astype(np.float64)
    sad = [(40 - (xx - 11.25) ** 2 + (yy - 12.375) ** 2 - 3 * (k - 2.125) ** 2).astype(np.float32) for k in range(5)]
    assert S.localise(sad, 0, 2, 12, 11, contrast=0.0, edge=1e9) is None


def _blob(size, cx, cy, sigma, ramp=0.0, theta=0.0):
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64)
    v = 60 + 150 * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * sigma ** 2))
    v += ramp * ((xx - cx) * math.cos(theta) + (yy - cy) * math.sin(theta))
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


def test_gaussian_blob_is_found_at_its_centre_and_scale():
    for sigma in (3.0, 5.0):
        img = _blob(128, 64.3, 60.7, sigma)
        kp, desc, total = S.extract(img)
        d = np.hypot(kp["x"] - 64.3, kp["y"] - 60.7)
        assert d.min() < 0.5, (sigma, d.min())
        best = kp[np.argmin(d)]
        assert abs(best["size"] - sigma) < 0.25 * sigma, (sigma, best["size"])


def test_orientation_follows_a_ramp_across_a_blob():
    for theta in (0.3, 2.0, 4.4):
        img = _blob(128, 64.0, 64.0, 4.0, ramp=3.0, theta=theta)
        kp, _, _ = S.extract(img)
        d = np.hypot(kp["x"] - 64.0, kp["y"] - 64.0)
        near = kp[d < 1.0]
        assert len(near) >= 1
        diff = np.abs((near["angle"] - theta + math.pi) % (2 * math.pi) - math.pi)
        assert diff.min() < math.radians(12), (theta, near["angle"])


def test_orientation_peaks_of_synthetic_histograms():
    h = np.zeros(36)
    h[10] = 1.0
    peaks = S.orientation_peaks(h)
    # the smoothed spike is symmetric about bin 10: angle exactly 10 bins
    assert len(peaks) == 1 and peaks[0][0] == 10 and abs(peaks[0][1] - 10 * 2 * math.pi / 36) < 1e-12
    h[30] = 0.85     # a second peak at 85 % of the first: kept; at 75 %: dropped
    assert [p[0] for p in S.orientation_peaks(h)] == [10, 30]
    h[30] = 0.75
    assert [p[0] for p in S.orientation_peaks(h)] == [10]
    # a peak at bin 0 with more weight on bin 35: the refined angle wraps below 2 pi
    h = np.zeros(36)
    h[0], h[35] = 1.0, 0.5
    (b, a), = S.orientation_peaks(h)
    assert b == 0 and 2 * math.pi - 0.2 < a < 2 * math.pi


def test_descriptor_norm_and_clip():
    img = _scene(129, 129, 30, 25, 21)
    kp, desc, total = S.extract(img)
    assert len(kp) > 10 and total == len(kp)
    v = desc.astype(np.float64)
    nrm = np.sqrt((v * v).sum(1))
    assert np.all(np.abs(nrm - 512) < 0.5 * math.sqrt(128) + 1)
    assert desc.max() <= 255
    # keypoints come octave by octave; one candidate's peaks in bin order
    assert np.all(np.diff(kp["octave"]) >= 0)
    # keeping fewer keeps the first ones
    kp2, desc2, total2 = S.extract(img, max_keypoints=7)
    assert total2 == total and np.array_equal(kp2, kp[:7]) and np.array_equal(desc2, desc[:7])


def test_rotation_by_90_degrees():
    """np.rot90 is an exact resampling; on a 129 x 129 image every octave has an odd size, so the
    subsampling commutes with it.  The blur's row-then-column order turns into column-then-row,
    which changes float32 rounding only: keypoints map onto rotated keypoints, angles turn by
    -pi/2 (rot90 turns the picture counter-clockwise, i.e. clockwise in y-down axes), and
    descriptors agree within rounding."""
    img = _scene(129, 129, 30, 25, 31)
    rot = np.ascontiguousarray(np.rot90(img))
    ka, da, _ = S.extract(img)
    kb, db, _ = S.extract(rot)
    # rot90: new (x', y') = (y, W - 1 - x)
    W = 129
    mapped_x, mapped_y = ka["y"], (W - 1) - ka["x"]
    found = 0
    for i in range(len(ka)):
        d = np.hypot(kb["x"] - mapped_x[i], kb["y"] - mapped_y[i])
        a = np.abs((kb["angle"] - (ka["angle"][i] - math.pi / 2) + math.pi) % (2 * math.pi) - math.pi)
        cand = np.nonzero((d < 1e-3) & (a < 1e-3) & (kb["octave"] == ka["octave"][i]))[0]
        if len(cand):
            found += 1
            j = cand[0]
            assert np.abs(db[j].astype(int) - da[i].astype(int)).max() <= 2
    assert len(ka) > 10 and found >= 0.9 * len(ka), (found, len(ka), len(kb))
