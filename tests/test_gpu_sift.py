"""GPU: SIFT extraction (xa_extract_sift) against the oracle (oracle/sift.py).

The scale space is the same bits on both sides (fp32 in one summation order) and the fit's
decisions are taken without division in one fp64 operation order, so the keypoint set,
octaves, layers, sample positions and orientation peaks are compared exactly.  Histograms are
summed in fixed point on the GPU (2^-40 and 2^-32 units) against fp64 sums in the oracle, and
the transcendental functions differ by an ulp or so: an orientation peak or an 8-bit descriptor
component can therefore differ only where the oracle's value sits within about 1e-9 of a
decision boundary.  The bars: identical keypoint keys (octave, layer, row, column, peak bin) in
the same order, positions / sizes / responses / angles within fp32 rounding of the oracle's
fp64 values, descriptor components within 1 and equal for at least 99.9 % of them."""
import sys

import numpy as np
import pytest

import synth
from oracle import geometry as OG
from oracle import match as OM
from oracle import sift as OS

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X.lib()
    return torch.device("cuda:0")


def _scene(w, h, n_blobs, n_rects, seed):
    sc = synth.make_scene(w, h, n_blobs, n_rects, seed)
    return synth.render(sc, np.eye(2), np.zeros(2), w, h, noise_seed=seed, supersample=2)


def _gpu(dev, img, **kw):
    t = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    kp, desc, count = X.extract_sift(t, X.sift_opts(**kw))
    torch.cuda.synchronize()
    c = count.cpu().numpy()
    n = int(c[0])
    return X.sift_keypoints_np(kp, n), desc[:n].cpu().numpy(), int(c[1])


def _compare(dev, img, label, **kw):
    gk, gd, gtot = _gpu(dev, img, **kw)
    ok, od, otot = OS.extract(img, **kw)
    say(f"[{label}] {img.shape[1]}x{img.shape[0]}: gpu {len(gk)} of {gtot}, oracle {len(ok)} of {otot}")
    assert gtot == otot and len(gk) == len(ok), label
    for f in ("octave", "layer", "xi", "yi", "peak"):
        assert np.array_equal(gk[f].astype(np.int64), ok[f].astype(np.int64)), (label, f)
    for f in ("x", "y", "size", "response"):
        err = np.abs(gk[f].astype(np.float64) - ok[f]) / np.maximum(np.abs(ok[f]), 1.0)
        assert err.max(initial=0) <= 2e-7, (label, f, err.max(initial=0))
    da = np.abs(gk["angle"].astype(np.float64) - ok["angle"])
    da = np.minimum(da, 2 * np.pi - da)
    assert da.max(initial=0) <= 1e-6, (label, da.max(initial=0))
    diff = np.abs(gd.astype(np.int64) - od.astype(np.int64))
    assert diff.max(initial=0) <= 1, label
    frac = float((diff != 0).mean()) if diff.size else 0.0
    assert frac <= 1e-3, (label, frac)
    say(f"[{label}] keys exact; descriptor components differing: {int((diff != 0).sum())} of {diff.size}")
    return gk, gd, gtot


def test_sift_small_scene(dev):
    say("case: 129x129 scene (odd octave sizes), default options")
    _compare(dev, _scene(129, 129, 30, 25, 31), "129 scene")


def test_sift_tiny_pair_images(dev):
    say("case: the tiny pair's images A (256x256) and B (its tilted view), 4096 keypoints at most")
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    _compare(dev, case.A, "tiny A")
    _compare(dev, case.B, "tiny B")


def test_sift_ragged_sizes_and_degenerate_images(dev):
    say("case: ragged 97x53, a constant image, images too small for a candidate row")
    _compare(dev, _scene(97, 53, 12, 10, 41), "97x53")
    for shape in ((64, 64), (10, 10), (11, 40), (1, 1)):
        k, d, tot = _gpu(dev, np.full(shape, 77, np.uint8))
        assert tot == 0 and len(k) == 0, shape
    # a single round blob on a small image (two octaves): its nearly flat orientation histogram
    # gives one keypoint per peak, five at one point
    yy, xx = np.mgrid[0:40, 0:40]
    blob = np.clip(60 + 150 * np.exp(-((xx - 19.6) ** 2 + (yy - 20.2) ** 2) / 18.0), 0, 255).astype(np.uint8)
    gk, _, _ = _compare(dev, blob, "40x40 blob")
    assert len(gk) == 5 and len(set(gk["peak"].tolist())) == 5


def test_sift_capacity_keeps_the_first(dev):
    say("case: max_keypoints below the number found keeps the first ones; a small raw capacity")
    img = _scene(129, 129, 30, 25, 31)
    gk, gd, tot = _gpu(dev, img, max_keypoints=7)
    ok, od, otot = OS.extract(img, max_keypoints=7)
    assert tot == otot and tot > 7 and len(gk) == 7
    assert np.array_equal(gk["xi"], ok["xi"]) and np.array_equal(gk["peak"].astype(int), ok["peak"])
    assert np.abs(gd.astype(int) - od.astype(int)).max() <= 1


def test_sift_full_size_image_and_determinism(dev):
    say("case: the full-size pair's image A (1024x768), twice (outputs identical run to run)")
    case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
    gk, gd, _ = _compare(dev, case.A, "full A")
    gk2, gd2, _ = _gpu(dev, case.A)
    assert np.array_equal(gk, gk2) and np.array_equal(gd, gd2)


def _oracle_kept_matches(kq, dq, kt, dt, num=3, den=4):
    """The oracle's kept L2 matches in query order: points (keypoint coordinates rounded to fp32
    as the GPU stores them), descriptor distances sqrt(d1^2)."""
    idx, d1, d2 = OM.nearest_two_l2(dq, dt)
    acc = OM.ratio_accept_l2(d1, d2, len(dt), num, den)
    pq = np.stack([kq["x"], kq["y"]], 1).astype(np.float32).astype(np.float64)[acc]
    pt = np.stack([kt["x"], kt["y"]], 1).astype(np.float32).astype(np.float64)[idx[acc]]
    return pq, pt, np.sqrt(d1[acc].astype(np.float64))


def test_sift_matches_and_eq1_against_the_oracle(dev):
    """Base-image selection of Sec. III.A on the tiny pair: the kept SIFT matches (points,
    distances) both ways and f1, f2 of eq. (1) equal the oracle's on its own SIFT output."""
    say("case: SIFT matches A -> B and B -> A of the tiny pair, eq. (1) both ways")
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    A, B = case.A, np.ascontiguousarray(case.B)
    ta, tb = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    fa, fb = X.sift_features(ta), X.sift_features(tb)
    ka, da, _ = OS.extract(A)
    kb, db, _ = OS.extract(B)
    fs = []
    for (fq, ft, kq, dq, kt, dt, lab) in ((fa, fb, ka, da, kb, db, "A->B"), (fb, fa, kb, db, ka, da, "B->A")):
        pq, pt, des, n = X.sift_match_points(fq, ft)
        torch.cuda.synchronize()
        n = int(n.item())
        rq, rt, rd = _oracle_kept_matches(kq, dq, kt, dt)
        assert n == len(rq) and n > 5, (lab, n, len(rq))
        assert np.array_equal(pq[:n].cpu().numpy(), rq) and np.array_equal(pt[:n].cpu().numpy(), rt), lab
        assert np.array_equal(des[:n].cpu().numpy(), rd), lab
        f = float(X.scaling_coefficient_f64(pq, pt, des, torch.tensor([n], dtype=torch.int32, device=dev)).item())
        rf = OG.scaling_coefficient(rq, rt, rd)
        assert abs(f - rf) <= 1e-9 * max(1.0, abs(rf)), (lab, f, rf)
        fs.append(f)
        say(f"[eq. 1 {lab}] {n} kept matches equal the oracle's; f = {f:.3f} (oracle {rf:.3f})")
    base, f1, f2 = X.select_base_image(ta, tb)
    assert (f1, f2) == (fs[0], fs[1]) and base == ("A" if fs[0] > fs[1] else "B")


def test_precise_stage_points_against_the_oracle(dev):
    """The precise stage's matches (Sec. III.C) on the tiny pair: SIFT of the oracle on the GPU's
    re-simulated views gives the same kept matches, taken back through the views' inverse maps."""
    say("case: precise stage matches on the re-simulated tiny pair against the oracle")
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    ta = torch.from_numpy(case.A).to(dev)
    tb = torch.from_numpy(np.ascontiguousarray(case.B)).to(dev)
    pa_par, pb_par = (2.0, 0.0, 0.0, 1.0, 0.0, 0.0), (1.0, 0.0, 0.0, 1.0, 0.0, 0.0)
    out = X.precise_stage(ta, tb, pa_par, pb_par, ransac_k=500)
    va, inv_a = X.simulated_view(ta, pa_par)
    vb, inv_b = X.simulated_view(tb, pb_par)
    ka, da, _ = OS.extract(va.cpu().numpy())
    kb, db, _ = OS.extract(vb.cpu().numpy())
    rq, rt, _ = _oracle_kept_matches(ka, da, kb, db)
    Ma, Mb = inv_a.reshape(2, 3), inv_b.reshape(2, 3)
    rq = rq @ Ma[:, :2].T + Ma[:, 2]
    rt = rt @ Mb[:, :2].T + Mb[:, 2]
    assert out["matches"] == len(rq)
    assert np.abs(out["pa"].cpu().numpy() - rq).max() <= 1e-9 and np.abs(out["pb"].cpu().numpy() - rt).max() <= 1e-9
    say(f"[precise] {out['matches']} matches equal the oracle's on the same views; {out['inliers']} inliers")
