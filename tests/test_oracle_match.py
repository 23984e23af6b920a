"""Pins of the oracle's matching, best pair and precision (Sec. III.B, Sec. IV.C, eqs. (5)-(6))."""
import numpy as np
import pytest

import synth
from oracle import match as M
from oracle import pipeline as PL
from oracle import plan as P


def _desc(seed, n):
    return np.random.default_rng(seed).integers(0, 256, (n, 32)).astype(np.uint8)


def _popcount_bruteforce(a, b):
    return sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b))


def test_hamming_matrix_brute_force():
    a, b = _desc(1, 13), _desc(2, 17)
    d = M.hamming_matrix(a, b)
    for i in range(13):
        for j in range(17):
            assert d[i, j] == _popcount_bruteforce(a[i], b[j])
    assert np.all(np.diag(M.hamming_matrix(a, a)) == 0)
    assert np.array_equal(M.hamming_matrix(a, b), M.hamming_matrix(b, a).T)


def test_nearest_two_brute_force():
    a, b = _desc(3, 25), _desc(4, 40)
    b[7] = b[3]                     # duplicated train descriptor
    a[5] = b[3]                     # query equal to both copies
    idx, d1, d2 = M.nearest_two(a, b)
    for q in range(25):
        ds = [_popcount_bruteforce(a[q], b[r]) for r in range(40)]
        m = min(ds)
        i = ds.index(m)
        assert (idx[q], d1[q]) == (i, m)
        assert d2[q] == min(ds[:i] + ds[i + 1:])
    assert (idx[5], d1[5], d2[5]) == (3, 0, 0)
    acc = M.ratio_accept(d1, d2, 40)
    assert not acc[5]               # equal distances never pass the ratio test


def test_ratio_test_is_exact():
    assert M.ratio_accept([4], [5], 2, 4, 5).tolist() == [False]     # 5*4 < 4*5 is false
    assert M.ratio_accept([3], [5], 2, 4, 5).tolist() == [True]
    assert M.ratio_accept([0], [9], 1, 4, 5).tolist() == [False]     # fewer than two train points


def test_empty_sets():
    idx, d1, d2 = M.nearest_two(np.zeros((0, 32), np.uint8), _desc(5, 4))
    assert idx.size == 0
    idx, d1, d2 = M.nearest_two(_desc(6, 3), np.zeros((0, 32), np.uint8))
    assert idx.tolist() == [-1] * 3 and d1.tolist() == [65535] * 3
    idx, d1, d2 = M.nearest_two(_desc(6, 3), _desc(7, 1))
    assert d2.tolist() == [65535] * 3


def test_best_pair_first_on_ties():
    a = [_desc(8, 10), _desc(9, 10)]
    b = [a[0].copy(), a[1].copy()]
    res, counts, best = M.match_views(a, b)
    assert counts[0] == counts[3] == 10
    assert best == (0, 0, 0, 10)


def test_precision_definition():
    pa = np.array([[1.0, 2.0], [10.0, 5.0], [3.0, 3.0]])
    H = np.array([[1.0, 0, 2.0], [0, 1.0, -1.0], [0, 0, 1.0]])
    pb = pa + np.array([2.0, -1.0])
    pb[2] += np.array([1.5, 1.5])                 # 2.12 px off
    frac, ok = M.precision(pa, pb, H, th=2.0)
    assert ok == 2 and frac == pytest.approx(2 / 3)
    assert M.precision(pa, pb, H, th=np.sqrt(8))[1] == 3


def test_tiny_pair_recovers_ground_truth():
    """End to end on a pair whose ground-truth map is known from rendering
    (tilt 2, rotation 30 deg): the best view pair's matches agree with it."""
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    grid = P.sampling_grid(2)
    opts = PL.OrbOptions(n_levels=3, n_features=300)
    out = PL.match_pair(case.A, case.B, grid, grid, opts, synth.brief_pattern())
    k, i, j, c = out["best"]
    assert c >= 40
    frac, ok = M.precision(out["pa"], out["pb"], case.H, 2.0)
    assert frac >= 0.8
    # the view pair that wins simulates (part of) the true tilt on the A side
    assert grid[i][0] > 1.0


# ------------------------------------------------------------------ L2 matching of SIFT descriptors

def test_l2sq_matrix_brute_force_and_scipy():
    from scipy.spatial.distance import cdist
    g = np.random.default_rng(41)
    Dq = g.integers(0, 256, (7, 128)).astype(np.uint8)
    Dt = g.integers(0, 256, (9, 128)).astype(np.uint8)
    d = M.l2sq_matrix(Dq, Dt)
    for i in range(7):
        for j in range(9):
            assert d[i, j] == sum((int(a) - int(b)) ** 2 for a, b in zip(Dq[i], Dt[j]))
    # squared Euclidean distances of 8-bit vectors stay far below 2^53: exact in fp64
    assert np.array_equal(d, cdist(Dq.astype(np.float64), Dt.astype(np.float64), "sqeuclidean").astype(np.int64))
    assert M.l2sq_matrix(np.full((1, 128), 255, np.uint8), np.zeros((1, 128), np.uint8))[0, 0] == 128 * 255 * 255


def test_nearest_two_l2_brute_force_ties_and_self():
    g = np.random.default_rng(42)
    Dt = g.integers(0, 40, (12, 128)).astype(np.uint8)
    Dt[7] = Dt[3]                                   # duplicate: equal distances go to the lower index
    Dq = np.concatenate([Dt[[3, 5]], g.integers(0, 40, (6, 128)).astype(np.uint8)])
    idx, d1, d2 = M.nearest_two_l2(Dq, Dt)
    for q in range(len(Dq)):
        ds = [sum((int(a) - int(b)) ** 2 for a, b in zip(Dq[q], Dt[r])) for r in range(len(Dt))]
        best = min(range(len(ds)), key=lambda r: (ds[r], r))
        assert idx[q] == best and d1[q] == ds[best]
        assert d2[q] == min(ds[r] for r in range(len(ds)) if r != best)
    assert idx[0] == 3 and d1[0] == 0 and d2[0] == 0 and not M.ratio_accept_l2(d1, d2, 12)[0]
    assert idx[1] == 5 and d1[1] == 0


def test_ratio_test_l2_is_exact_on_squared_distances():
    # d1 / d2 = 3 / 4 exactly (squared 9 : 16) is rejected; just below is accepted
    d1 = np.array([9, 9 * 10000 - 1, 0, 5])
    d2 = np.array([16, 16 * 10000, 0, M.L2_MISSING])
    acc = M.ratio_accept_l2(d1, d2, 2, 3, 4)
    assert acc.tolist() == [False, True, False, True]
    assert not M.ratio_accept_l2(d1, d2, 1, 3, 4).any()


def test_l2_missing_neighbours():
    D = np.zeros((3, 128), np.uint8)
    idx, d1, d2 = M.nearest_two_l2(D, D[:0])
    assert (idx == -1).all() and (d1 == M.L2_MISSING).all() and (d2 == M.L2_MISSING).all()
    idx, d1, d2 = M.nearest_two_l2(D, D[:1])
    assert (idx == 0).all() and (d1 == 0).all() and (d2 == M.L2_MISSING).all()
