"""GPU: the precise stage after the search — best-pair points, homography RANSAC with
caller-drawn samples and the inlier share of eq. (7) — against the oracle."""
import sys

import numpy as np
import pytest

import synth
from oracle import geometry as OG
from oracle import match as OM
from oracle import orb as OO
from oracle import pipeline as OPL
from oracle import plan as OP
from oracle import simulate as OS

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X.lib()
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _Ht():
    return np.array([[0.9, 0.2, 15.0], [-0.1, 1.1, -7.0], [2e-4, -1e-4, 1.0]])


def _apply(H, p):
    q = np.c_[p, np.ones(len(p))] @ H.T
    return q[:, :2] / q[:, 2:]


def test_ransac_matches_the_oracle(dev):
    say("case: RANSAC on 400 matches (30% outliers), 600 samples incl. degenerate and out-of-range ones")
    g = synth.rng(41)
    n = 400
    pa = g.uniform(0, 900, (n, 2))
    pb = _apply(_Ht(), pa) + g.normal(0, 0.8, (n, 2))
    bad = g.choice(n, 120, replace=False)
    pb[bad] = g.uniform(0, 900, (120, 2))
    pa[20] = pa[3] + 2.5 * (pa[7] - pa[3])                  # 3, 7, 20 collinear -> a degenerate sample
    samples = X.draw_samples(n, 600, seed=3)
    samples[10] = [3, 7, 20, 30]
    samples[11] = [0, 1, 2, n]                              # out of range -> -1
    th = 3.0
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    scores, best, H, inl = X.ransac_homography(t(pa), t(pb), t(samples), th)
    torch.cuda.synchronize()
    scores, best, H, inl = scores.cpu().numpy(), best.cpu().numpy(), H.cpu().numpy(), inl.cpu().numpy()
    ok = samples[:, :].max(axis=1) < n
    rs, rb, rH, rinl = OG.ransac(pa, pb, np.where(ok[:, None], samples, 0), th)
    rs = np.where(ok, rs, -1)
    # a score may differ only when some residual sits within 1e-6 px of the threshold
    diff = np.flatnonzero(scores != rs)
    for k in diff:
        Hk = OG.homography_from_4(pa[samples[k]], pb[samples[k]])
        assert Hk is not None and np.min(np.abs(OG.residuals(Hk, pa, pb) - th)) < 1e-6, k
    assert scores[10] == -1 and scores[11] == -1
    assert best[0] == rb and best[1] == rs[rb]
    # the refit: fixed-order normal equations on the GPU, an SVD least-squares solve in the oracle
    assert np.abs(H - rH).max() <= 1e-7 * np.abs(rH).max()
    amb = np.abs(OG.residuals(rH, pa, pb) - th) < 1e-6
    assert np.array_equal(inl.astype(bool) | amb, rinl | amb)
    say(f"[ransac] best sample {best.tolist()}, {int(inl.sum())} inliers of {n}; scores equal on "
        f"{len(scores) - len(diff)}/{len(scores)}")


def test_ransac_empty_inputs(dev):
    z = torch.zeros((0, 2), dtype=torch.float64, device=dev)
    s = torch.zeros((0, 4), dtype=torch.int32, device=dev)
    scores, best, H, inl = X.ransac_homography(z, z, s, 2.0)
    torch.cuda.synchronize()
    assert best.cpu().tolist() == [-1, -1] and float(H.abs().max()) == 0.0


def test_best_pair_points_equal_the_oracle(dev):
    """ORB and matching on the oracle's views are exact, so the best pair's accepted matches in
    original coordinates equal the oracle's (same order, 1e-9 px)."""
    say("case: best-pair points from GPU ORB + matching on the oracle's views of the tiny pair")
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    B = np.ascontiguousarray(case.B)
    grid = OP.sampling_grid(1)
    opts = OPL.OrbOptions(n_levels=3, n_features=300)
    pat = synth.brief_pattern()
    ref = OPL.match_pair(case.A, B, grid, grid, opts, pat)
    params = X.make_params([(t, f) for t, f in grid])
    feats = []
    for img, views in ((case.A, ref["views_a"]), (B, ref["views_b"])):
        plan = X.plan_image(img.shape[1], img.shape[0], params, 3, 1.2, 300, 20)
        arena = np.zeros(plan.arena_bytes, np.uint8)
        mask = np.zeros(plan.arena_bytes, np.uint8)
        for i, v in enumerate(views):
            V, M, U = OS.simulate_view(img, v)
            plan.level_image(arena, i, 0)[:] = U
            plan.level_image(mask, i, 0)[:] = M.astype(np.uint8)
        feats.append(X.extract_orb(plan, torch.from_numpy(arena).to(dev), torch.from_numpy(mask).to(dev),
                                   torch.from_numpy(pat).to(dev)))
    (kpa, da, ca), (kpb, db, cb) = feats
    m, pc, best = X.match_views(da, ca, db, cb)
    pa, pb, dist, n = X.best_pair_points(kpa, kpb, m, ca, cb, best, len(grid), 300)
    torch.cuda.synchronize()
    n = int(n.item())
    assert tuple(best.cpu().tolist()) == tuple(ref["best"])
    assert n == len(ref["pa"]) == int(ref["best"][3])
    assert np.allclose(pa[:n].cpu().numpy(), ref["pa"], atol=1e-9, rtol=0)
    assert np.allclose(pb[:n].cpu().numpy(), ref["pb"], atol=1e-9, rtol=0)
    k, i, j, c = ref["best"]
    idx, d1, d2, acc = ref["results"][k]
    assert np.array_equal(dist[:n].cpu().numpy(), d1[acc])
    # eq. (1) on these matches equals the oracle's
    f = float(X.scaling_coefficient(pa, pb, dist, torch.tensor([n], dtype=torch.int32, device=dev)).item())
    rf = OG.scaling_coefficient(ref["pa"], ref["pb"], d1[acc])
    assert abs(f - rf) <= 1e-9 * max(1.0, abs(rf))
    say(f"[pair points] {n} accepted matches equal the oracle's; eq. (1) f = {f:.4f}")


def test_precise_stage_recovers_the_ground_truth(dev):
    """Re-simulation at the true view (tilt 2 along phi = 0 for A, identity for B), SIFT, L2
    matching and RANSAC on the tiny pair: H maps A's corners within 2 px of the ground truth and
    the inlier share of eq. (7) is high."""
    say("case: precise stage (Lanczos re-simulation, SIFT, RANSAC) on the tiny pair")
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    A = torch.from_numpy(case.A).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(case.B)).to(dev)
    out = X.precise_stage(A, B, (2.0, 0.0, 0.0, 1.0, 0.0, 0.0), (1.0, 0.0, 0.0, 1.0, 0.0, 0.0), ransac_k=1000,
                          th=3.0)
    corners = np.array([[0.0, 0.0], [255.0, 0.0], [0.0, 255.0], [255.0, 255.0], [128.0, 128.0]])
    err = np.linalg.norm(_apply(out["H"], corners) - _apply(case.H, corners), axis=1)
    say(f"[precise] {out['matches']} matches, {out['inliers']} inliers (eq. 7: {out['inlier_ratio']:.3f}); "
        f"corner error {err.max():.2f} px")
    assert out["matches"] > 20 and out["inlier_ratio"] >= 0.8 and err.max() <= 2.0
    # the oracle's RANSAC on the same points and samples agrees
    pa, pb = out["pa"].cpu().numpy(), out["pb"].cpu().numpy()
    rs, rb, rH, rinl = OG.ransac(pa, pb, out["samples"].cpu().numpy(), 3.0)
    assert rs[rb] == out["inliers"]
    assert np.abs(out["H"] - rH).max() <= 1e-7 * np.abs(rH).max()


def test_base_image_selection_prefers_the_closer_view(dev):
    """Eq. (1) both ways on SIFT matches of a pair where B is A's scene seen from twice the
    distance (every length halves): A is the base (f1 > 0 > f2)."""
    say("case: base-image selection (eq. (1)) on a pair with a 2x scale change")
    sc = synth.make_scene(512, 512, 160, 120, 77)
    A = synth.render(sc, np.eye(2), np.zeros(2), 512, 512, noise_seed=1)
    B = synth.render(sc, 0.5 * np.eye(2), np.zeros(2), 256, 256, noise_seed=2)
    base, f1, f2 = X.select_base_image(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev))
    say(f"[base image] {base}: f1 = {f1:.1f}, f2 = {f2:.1f}")
    assert base == "A" and f1 > 0 > f2
