"""GPU: the L2 matcher of 8-bit SIFT descriptors (xa_match_l2, int8 matrix cores) against the
oracle's exact squared distances, nearest two (lowest index on ties) and ratio test, bit for bit."""
import sys

import numpy as np
import pytest

import synth
from oracle import match as OM

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


def _run(dev, Q, T, num=3, den=4):
    q = torch.from_numpy(np.ascontiguousarray(Q, np.uint8).reshape(-1, 128)).to(dev)
    t = torch.from_numpy(np.ascontiguousarray(T, np.uint8).reshape(-1, 128)).to(dev)
    out, count = X.match_l2(q, t, num, den)
    torch.cuda.synchronize()
    return X.l2_matches_np(out), int(count.cpu()[0])


def _check(dev, Q, T, label, num=3, den=4, sample=None):
    g, cnt = _run(dev, Q, T, num, den)
    assert len(g) == len(Q)
    rows = np.arange(len(Q)) if sample is None else np.asarray(sample)
    idx, d1, d2 = OM.nearest_two_l2(Q[rows], T)
    assert np.array_equal(g["t"][rows].astype(np.int64), idx), label
    assert np.array_equal(g["d1"][rows].astype(np.int64), d1), label
    assert np.array_equal(g["d2"][rows].astype(np.int64), d2), label
    acc = OM.ratio_accept_l2(d1, d2, len(T), num, den)
    if sample is None:
        assert cnt == int(acc.sum()), label
    else:   # every query decided on the GPU's own distances, which equal the oracle's on the sample
        gacc = OM.ratio_accept_l2(g["d1"].astype(np.int64), g["d2"].astype(np.int64), len(T), num, den)
        assert cnt == int(gacc.sum()), label
    say(f"[{label}] {len(Q)} x {len(T)}: exact on {len(rows)} queries, {cnt} pass the ratio test")
    return g, cnt


def test_l2_random_sets_ragged(dev):
    say("case: SIFT-like sets 300 x 517 (3 query blocks, 5 chunks with a ragged tail), ratios 3/4 and 4/5")
    Q, T, src = synth.sift_like_sets(300, 517, 11)
    g, cnt = _check(dev, Q, T, "ragged 3/4")
    _check(dev, Q, T, "ragged 4/5", 4, 5)
    ok = OM.ratio_accept_l2(g["d1"].astype(np.int64), g["d2"].astype(np.int64), len(T))
    assert cnt > 50 and (g["t"][ok] == src[ok]).mean() > 0.95


def test_l2_many_train_slices(dev):
    say("case: 70 queries x 20000 train (one query block, 157 train slices merged per query)")
    Q, T, _ = synth.sift_like_sets(70, 20000, 12)
    _check(dev, Q, T, "many slices")


def test_l2_duplicates_self_matches_and_ties(dev):
    say("case: duplicated train rows (ties go to the lower index, d2 = d1) and queries equal to train rows")
    g0 = np.random.default_rng(13)
    T = synth.sift_like_descriptors(400, 13)
    T[[50, 200, 399]] = T[10]                       # four equal rows
    T[130] = T[129]
    Q = np.concatenate([T[[10, 129, 200, 5]], synth.sift_like_descriptors(60, 14)])
    Q = np.concatenate([Q, np.clip(T[g0.integers(0, 400, 40)].astype(int) + g0.integers(-2, 3, (40, 128)), 0, 255)])
    Q = Q.astype(np.uint8)
    g, _ = _check(dev, Q, T, "duplicates")
    assert g["t"][0] == 10 and g["d1"][0] == 0 and g["d2"][0] == 0
    assert g["t"][1] == 129 and g["d2"][1] == 0


def test_l2_extreme_components(dev):
    say("case: components at 0 and 255 (the int8 centring at both ends, the largest distance 128 * 255^2)")
    g0 = np.random.default_rng(15)
    T = (g0.integers(0, 2, (97, 128)) * 255).astype(np.uint8)
    T[0] = 0
    T[1] = 255
    Q = (g0.integers(0, 2, (65, 128)) * 255).astype(np.uint8)
    Q[0] = 255
    Q[1] = 0
    Q[2] = np.where(np.arange(128) % 2 == 0, 0, 255)
    g, _ = _check(dev, Q, T, "extremes")
    assert g["d1"][0] == 0 and g["t"][0] == 1
    s = OM.l2sq_matrix(Q[:1], T[:1])[0, 0]
    assert s == 128 * 255 * 255


def test_l2_empty_and_single(dev):
    say("case: empty train, one train row, empty and single query sets")
    Q, T, _ = synth.sift_like_sets(33, 1, 16)
    _check(dev, Q, T, "one train row")
    g, cnt = _run(dev, Q, T[:0])
    assert (g["t"] == -1).all() and (g["d1"] == X.L2_MISSING).all() and (g["d2"] == X.L2_MISSING).all() and cnt == 0
    g, cnt = _run(dev, Q[:0], T)
    assert len(g) == 0 and cnt == 0
    _check(dev, Q[:1], synth.sift_like_descriptors(300, 17), "single query")


def test_l2_at_4096_sampled(dev):
    say("case: 4096 x 4096 (the size the benchmark times is larger; 256 queries checked)")
    Q, T, _ = synth.sift_like_sets(4096, 4096, 18)
    sample = np.random.default_rng(19).choice(4096, 256, replace=False)
    _check(dev, Q, T, "4096 sampled", sample=np.sort(sample))
