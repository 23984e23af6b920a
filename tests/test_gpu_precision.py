"""GPU: the precision of eqs. (5)-(6) (xa_pair_precision) against the oracle on the same matches.

The GPU's best view pair is turned into point pairs by xa_best_pair_points, and the oracle's
precision is evaluated on exactly those points.  The kernel's (correct, accepted) must equal the
oracle's count, except for matches whose oracle error lies within AMBIGUITY px of the threshold
(there the two evaluations of |H p_a - p_b| may round to opposite sides; both are taken without
fused multiply-adds, so in practice the band is empty).  Cases: the tiny pair, the full-size pair
(45 views per image, 1000 keypoints), and hand-placed keypoints whose errors sit exactly at, just
above and just below the threshold under a projective H."""
import sys

import numpy as np
import pytest

import synth
from oracle import match as OM
from oracle import plan as OP

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu

TH = 2.0
AMBIGUITY = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X.lib()
    return torch.device("cuda:0")


def _oracle_errors(pa, pb, H):
    h = np.concatenate([pa, np.ones((pa.shape[0], 1))], axis=1) @ np.asarray(H, np.float64).T
    proj = h[:, :2] / h[:, 2:3]
    return np.sqrt(((proj - pb) ** 2).sum(axis=1))


def _check_run(run, H, n_b, N, label):
    pr = run.precision(H, TH).cpu().numpy()
    pa, pb, _, n = X.best_pair_points(run.kp_a, run.kp_b, run.matches, run.count_a, run.count_b, run.best, n_b, N)
    n = int(n.item())
    pa = pa[:n].cpu().numpy()
    pb = pb[:n].cpu().numpy()
    frac, ok = OM.precision(pa, pb, H, TH)
    band = int((np.abs(_oracle_errors(pa, pb, H) - TH) <= AMBIGUITY).sum()) if n else 0
    say(f"[{label}] gpu {pr.tolist()} oracle {ok}/{n} (band {band})")
    assert pr[1] == n == int(run.best[3].item())
    assert abs(int(pr[0]) - ok) <= band
    return pr


def _pair_run(dev, case, n_tilt, levels, N):
    grid = OP.sampling_grid(n_tilt)
    params = X.make_params([(t, f) for t, f in grid])
    pa = X.plan_image(case.A.shape[1], case.A.shape[0], params, levels, 1.2, N, 20)
    pb = X.plan_image(case.B.shape[1], case.B.shape[0], params, levels, 1.2, N, 20)
    run = X.PairRunner(pa, pb, dev)
    run.run(torch.from_numpy(np.ascontiguousarray(case.A)).to(dev),
            torch.from_numpy(np.ascontiguousarray(case.B)).to(dev), torch.from_numpy(synth.brief_pattern()).to(dev))
    return run, len(grid)


def test_precision_tiny_pair(dev):
    say("case: precision of the tiny pair's best view pair against the oracle on the same points")
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    run, nv = _pair_run(dev, case, 2, 3, 300)
    pr = _check_run(run, case.H, nv, 300, "tiny")
    assert pr[1] >= 40


def test_precision_full_pair(dev):
    say("case: precision of the full-size pair's best view pair against the oracle on the same points")
    case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
    run, nv = _pair_run(dev, case, 5, 8, 1000)
    pr = _check_run(run, case.H, nv, 1000, "full")
    assert pr[1] >= 100


def test_precision_hand_placed(dev):
    """Errors of exactly th, one ulp above and below, under H = 2 x a translation (w = 2)."""
    say("case: hand-placed matches at the precision threshold")
    N = 8
    H = np.array([[2.0, 0.0, 10.0], [0.0, 2.0, -6.0], [0.0, 0.0, 2.0]])   # (x, y) -> (x + 5, y - 3)
    a_pts = [(10.0, 20.0), (33.5, 7.25), (100.0, 40.0), (4.0, 4.0), (50.0, 50.0), (60.0, 61.0), (0.0, 0.0)]
    # H p_a = (x + 5, y - 3); b at distance exactly th, one ulp beyond, one ulp inside, 1.5, 0 and 5
    b_pts = [(17.0, 17.0), (38.5, 2.25), (np.nextafter(107.0, 200.0), 37.0), (9.0, np.nextafter(3.0, 0.0)),
             (56.5, 47.0), (65.0, 58.0), (8.0, 1.0)]
    kp_a = np.zeros((1, N), X.KEYPOINT_DTYPE)
    kp_b = np.zeros((1, N), X.KEYPOINT_DTYPE)
    m = np.zeros((1, N), X.MATCH_DTYPE)
    for q, ((x, y), (bx, by)) in enumerate(zip(a_pts, b_pts)):
        kp_a[0, q]["xs"], kp_a[0, q]["ys"] = x, y
        t = len(a_pts) - 1 - q                       # matches in reverse train order
        kp_b[0, t]["xs"], kp_b[0, t]["ys"] = bx, by
        m[0, q] = (t, 10, 40)                        # accepted: 5 * 10 < 4 * 40
    m[0, 6]["d1"] = 32                               # 5 * 32 < 4 * 40 fails: not accepted
    # the train view holds 7 keypoints, the query view 7; entry 7 is beyond both counts
    m[0, 7] = (0, 0, 100)

    def dev_bytes(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).reshape(a.shape[0], N, -1)).to(dev)

    ka, kb, mm = dev_bytes(kp_a), dev_bytes(kp_b), dev_bytes(m)
    ca = torch.tensor([7], dtype=torch.int32, device=dev)
    cb = torch.tensor([7], dtype=torch.int32, device=dev)
    best = torch.tensor([0, 0, 0, 6], dtype=torch.int32, device=dev)
    out = torch.zeros(2, dtype=torch.int32, device=dev)
    Hc = np.ascontiguousarray(H, np.float64).reshape(9)
    X._check(X.lib().xa_pair_precision(X._ptr(ka), X._ptr(kb), X._ptr(mm), X._ptr(ca), X._ptr(cb), 1, N, 4, 5,
                                       X._ptr(best), Hc.ctypes.data, TH, X._ptr(out), X._stream()))
    got = out.cpu().numpy()
    # oracle on the accepted matches (queries 0..5)
    pa = np.array(a_pts[:6])
    pb = np.array(b_pts[:6])
    frac, ok = OM.precision(pa, pb, H, TH)
    say(f"[hand-placed] gpu {got.tolist()} oracle {ok}/6")
    # at th exactly, below it and inside: correct; one ulp above: not
    assert ok == 5 and got.tolist() == [5, 6]
    # an invalid best pair counts nothing
    best_bad = torch.tensor([-1, -1, -1, 0], dtype=torch.int32, device=dev)
    X._check(X.lib().xa_pair_precision(X._ptr(ka), X._ptr(kb), X._ptr(mm), X._ptr(ca), X._ptr(cb), 1, N, 4, 5,
                                       X._ptr(best_bad), Hc.ctypes.data, TH, X._ptr(out), X._stream()))
    assert out.cpu().numpy().tolist() == [0, 0]
