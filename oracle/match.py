"""Brute-force Hamming matching, ratio test, best view pair, back-mapping and precision.

Test infrastructure only (see the package docstring).

Sec. III.B matches every simulated image with a brute-force Hamming matcher
and keeps the parameters of the view with the most matches; Sec. IV.C screens
matches with a nearest / second-nearest distance ratio.  Precision follows
eqs. (5)-(6): a match is correct when the ground-truth map sends the first
point within Th pixels of its match.

Parity status: pinned (a pure-Python popcount brute force, d(x, x) = 0,
symmetry, duplicated train descriptors force d2 = d1 and reject; for the L2 matcher of SIFT
descriptors a pure-Python brute force of the squared distances, scipy's squared-Euclidean
distance, the exact ratio boundary and the missing-neighbour cases).
"""
from __future__ import annotations

import numpy as np


def hamming_matrix(Dq, Dt):
    """d[q, r] = popcount(Dq[q] xor Dt[r]) over 256-bit descriptors (n x 32 u8)."""
    a = np.ascontiguousarray(Dq, np.uint8).view(np.uint64)        # (nq, 4)
    b = np.ascontiguousarray(Dt, np.uint8).view(np.uint64)        # (nt, 4)
    return np.bitwise_count(a[:, None, :] ^ b[None, :, :]).sum(axis=2, dtype=np.int64)


def nearest_two(Dq, Dt):
    """For each query: idx1 = smallest train index attaining the minimum distance d1;
    d2 = minimum over the other train descriptors (may equal d1).
    Missing values (fewer than 1 or 2 train descriptors) are -1 / 65535."""
    nq, nt = len(Dq), len(Dt)
    idx = np.full(nq, -1, np.int64)
    d1 = np.full(nq, 65535, np.int64)
    d2 = np.full(nq, 65535, np.int64)
    if nq == 0 or nt == 0:
        return idx, d1, d2
    d = hamming_matrix(Dq, Dt)
    idx = np.argmin(d, axis=1)                      # first minimum = smallest index
    d1 = d[np.arange(nq), idx]
    if nt >= 2:
        d[np.arange(nq), idx] = 1 << 30
        d2 = d.min(axis=1)
    return idx.astype(np.int64), d1, d2


def ratio_accept(d1, d2, n_train: int, num: int = 4, den: int = 5):
    """Accept iff there are at least two train descriptors and d1 < (num/den) d2,
    evaluated exactly as den * d1 < num * d2."""
    d1 = np.asarray(d1, np.int64)
    d2 = np.asarray(d2, np.int64)
    if n_train < 2:
        return np.zeros(d1.shape, bool)
    return den * d1 < num * d2


# ------------------------------------------------------------------ L2 matching of SIFT descriptors
# Sec. III.A and III.C match SIFT descriptors (128-D) by descriptor distance with the same
# nearest / second-nearest screening (threshold 0.75, Sec. IV.C).  Reading: the descriptor is
# in its usual 8-bit quantised form (components 0..255) and the distance is Euclidean; ranking
# by the squared distance is the same, and the ratio test d1 < (num/den) d2 on distances is
# den^2 d1^2 < num^2 d2^2 on squared ones, exact in integers.

L2_MISSING = (1 << 32) - 1          # squared distance reported where a neighbour does not exist


def l2sq_matrix(Dq, Dt):
    """d[q, r] = sum_k (Dq[q, k] - Dt[r, k])^2 (int64, exact)."""
    a = np.asarray(Dq, np.int64)
    b = np.asarray(Dt, np.int64)
    return (a * a).sum(axis=1)[:, None] + (b * b).sum(axis=1)[None, :] - 2 * (a @ b.T)


def nearest_two_l2(Dq, Dt):
    """For each query: idx1 = smallest train index attaining the minimum squared distance d1;
    d2 = minimum over the other train descriptors (may equal d1).  Missing values are
    -1 / L2_MISSING."""
    nq, nt = len(Dq), len(Dt)
    idx = np.full(nq, -1, np.int64)
    d1 = np.full(nq, L2_MISSING, np.int64)
    d2 = np.full(nq, L2_MISSING, np.int64)
    if nq == 0 or nt == 0:
        return idx, d1, d2
    d = l2sq_matrix(Dq, Dt)
    idx = np.argmin(d, axis=1)                      # first minimum = smallest index
    d1 = d[np.arange(nq), idx]
    if nt >= 2:
        d[np.arange(nq), idx] = np.iinfo(np.int64).max
        d2 = d.min(axis=1)
    return idx.astype(np.int64), d1, d2


def ratio_accept_l2(d1sq, d2sq, n_train: int, num: int = 3, den: int = 4):
    """Accept iff there are at least two train descriptors and d1 < (num/den) d2 on distances,
    evaluated exactly on squared distances as den^2 d1^2 < num^2 d2^2."""
    d1sq = np.asarray(d1sq, np.int64)
    d2sq = np.asarray(d2sq, np.int64)
    if n_train < 2:
        return np.zeros(d1sq.shape, bool)
    return den * den * d1sq < num * num * d2sq


def match_views(descs_a, descs_b, num: int = 4, den: int = 5, pairs=None):
    """Match the views of image A (queries) against the views of image B (train).

    pairs: iterable of (i, j), default the full cross product in row-major
    order.  Returns (results, counts, best) where results[k] = (idx, d1, d2,
    accepted) for pair k, counts[k] = number of accepted queries, and best =
    (k, i, j, count) of the pair with the most matches, the first such pair
    in pair order on ties."""
    if pairs is None:
        pairs = [(i, j) for i in range(len(descs_a)) for j in range(len(descs_b))]
    results, counts = [], []
    for (i, j) in pairs:
        idx, d1, d2 = nearest_two(descs_a[i], descs_b[j])
        acc = ratio_accept(d1, d2, len(descs_b[j]), num, den)
        results.append((idx, d1, d2, acc))
        counts.append(int(acc.sum()))
    counts = np.asarray(counts, np.int64)
    if len(pairs) == 0:
        return results, counts, (-1, -1, -1, 0)
    k = int(np.argmax(counts))
    return results, counts, (k, pairs[k][0], pairs[k][1], int(counts[k]))


def level_to_view(x, y, level_w: int, level_h: int, w0: int, h0: int):
    """Level pixel -> view (level 0) pixel: x0 = (x + 1/2) W0 / W_l - 1/2 (likewise y)."""
    return ((np.asarray(x, np.float64) + 0.5) * (w0 / level_w) - 0.5,
            (np.asarray(y, np.float64) + 0.5) * (h0 / level_h) - 0.5)


def view_to_source(view, x, y):
    """p = G(q) with the view's inverse map."""
    G = view.inv
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return G[0, 0] * x + G[0, 1] * y + G[0, 2], G[1, 0] * x + G[1, 1] * y + G[1, 2]


def precision(pa, pb, H, th: float = 2.0):
    """Eqs. (5)-(6): fraction of matches (pa -> pb) whose ground-truth image H pa
    lies within th pixels of pb.  H is 3x3 acting on homogeneous coordinates."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    if pa.shape[0] == 0:
        return 0.0, 0
    h = np.concatenate([pa, np.ones((pa.shape[0], 1))], axis=1) @ np.asarray(H, np.float64).T
    proj = h[:, :2] / h[:, 2:3]
    err = np.sqrt(((proj - pb) ** 2).sum(axis=1))
    ok = int((err <= th).sum())
    return ok / pa.shape[0], ok
