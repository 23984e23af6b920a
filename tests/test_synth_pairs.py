"""The pair generator's ground-truth map, pinned by the rendered pixels rather than by the
formula that builds it: image B resampled at H(p) for the pixels p of image A reproduces A
(both images see the same scene through their own affine maps), and a map that ignores A's own
tilt does not.  H is what the precision of eqs. (5)-(6) is scored against."""
import math

import numpy as np
from scipy import ndimage

import synth


def _agreement(A, B, H):
    ya, xa = np.mgrid[0:A.shape[0], 0:A.shape[1]].astype(np.float64)
    xb = H[0, 0] * xa + H[0, 1] * ya + H[0, 2]
    yb = H[1, 0] * xa + H[1, 1] * ya + H[1, 2]
    inside = (xb >= 0) & (xb <= B.shape[1] - 1) & (yb >= 0) & (yb <= B.shape[0] - 1)
    vb = ndimage.map_coordinates(B.astype(np.float64), [yb[inside], xb[inside]], order=1)
    va = A.astype(np.float64)[inside]
    return float(np.corrcoef(va, vb)[0, 1]), float(np.mean(np.abs(va - vb))), int(inside.sum())


def test_two_tilt_pair_map_follows_the_content():
    # A tilted by 1.6 along longitude 0.3 rad, B by 2 along y: the map from A to B has both tilts
    case = synth.make_pair(320, 240, 60, 0, 9, t=2.0, phi=math.pi / 2, psi=-math.pi / 2,
                           t_a=1.6, phi_a=0.3)
    r, mad, n = _agreement(case.A, case.B, case.H)
    assert n > 0.5 * case.A.size
    assert r > 0.97 and mad < 4.0, (r, mad)
    # the map of a head-on A (B's own transform) is wrong for this pair
    M = synth.tilt_rotation(2.0, math.pi / 2, -math.pi / 2)
    _, _, off = synth.affine_canvas(M, 320, 240)
    Hw = np.eye(3)
    Hw[:2, :2] = M
    Hw[:2, 2] = off
    rw, _, _ = _agreement(case.A, case.B, Hw)
    assert rw < r - 0.3, (r, rw)


def test_head_on_pair_unchanged():
    # t_a = 1 keeps A the head-on scene and H the transform of B
    case = synth.make_pair(200, 150, 30, 10, 5, t=2.5, phi=0.4, psi=0.7)
    M = synth.tilt_rotation(2.5, 0.4, 0.7)
    bw, bh, off = synth.affine_canvas(M, 200, 150)
    assert case.A.shape == (150, 200) and case.B.shape == (bh, bw)
    assert np.array_equal(case.H[:2, :2], M) and np.allclose(case.H[:2, 2], off, atol=1e-12)
    r, mad, _ = _agreement(case.A, case.B, case.H)
    assert r > 0.97 and mad < 4.0, (r, mad)


def test_stress_configuration_geometry():
    # both images under absolute tilt 80 deg in orthogonal directions: transition tilt t^2
    cfg = synth.PAIR_CONFIGS["stress"]
    t = 1.0 / math.cos(math.radians(80.0))
    MA = synth.tilt_rotation(cfg["t_a"], cfg["phi_a"], 0.0)
    MB = synth.tilt_rotation(cfg["t"], cfg["phi"], cfg["psi"])
    assert np.allclose(MA, np.diag([1.0 / t, 1.0]), atol=1e-12)
    assert np.allclose(MB, np.diag([1.0, 1.0 / t]), atol=1e-12)
    sv = np.linalg.svd(MB @ np.linalg.inv(MA), compute_uv=False)
    assert abs(sv[0] / sv[1] - t * t) < 1e-9 and abs(math.degrees(math.acos(1.0 / (t * t))) - 88.27) < 0.01
    assert synth.affine_canvas(MA, 4096, 3072)[:2] == (712, 3072)
    assert synth.affine_canvas(MB, 4096, 3072)[:2] == (4096, 534)
