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
