"""Homography RANSAC over matched points, the inlier ratio of eq. (7), and the scaling
coefficient of eq. (1) that picks the base image.

Test infrastructure only (see the package docstring).

Sec. III.C screens the final matches with RANSAC on a homography; eq. (7) scores a
method by the share of matched points that RANSAC keeps as inliers.  Here the random
draws are an input (K samples of 4 match indices), so the result is a plain function
of the points, the samples and the threshold:

* a sample is degenerate iff some 3 of its 4 points, in image A or in image B, span a
  doubled triangle area |cross| < 1 px^2 (then it scores -1);
* otherwise H (3x3, h33 = 1) is the solution of the 8x8 linear system that maps the 4
  points of A onto those of B (numpy.linalg.solve);
* its score is the number of matches with |H(p_a) - p_b| <= th, H(p) the projective
  image (u/w, v/w); a match with w <= 0 is an outlier;
* the best sample has the highest score, the lowest index on ties (none if every
  sample is degenerate); its inliers are refitted by least squares in Hartley-normalised
  coordinates.

Parity status: pinned.  The solved H maps its 4 points exactly onto their targets and
recovers a known homography from any 4 of its correspondences; degenerate samples
score -1; on data with a known homography and gross outliers the best score equals
the number of true inliers and the refit recovers the homography; the refit of exact
correspondences is exact; the inlier ratio is the plain quotient of eq. (7).
"""
from __future__ import annotations

import numpy as np

DEGENERATE_AREA = 1.0          # doubled triangle area (px^2) below which 3 points count as collinear


def degenerate(p4) -> bool:
    """Some 3 of the 4 points (4 x 2) span |cross| < DEGENERATE_AREA."""
    p = np.asarray(p4, np.float64)
    for a, b, c in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
        cross = (p[b, 0] - p[a, 0]) * (p[c, 1] - p[a, 1]) - (p[b, 1] - p[a, 1]) * (p[c, 0] - p[a, 0])
        if abs(cross) < DEGENERATE_AREA:
            return True
    return False


def homography_from_4(src4, dst4):
    """H with h33 = 1 mapping the 4 src points onto the 4 dst points, or None if degenerate."""
    s = np.asarray(src4, np.float64)
    d = np.asarray(dst4, np.float64)
    if degenerate(s) or degenerate(d):
        return None
    A = np.zeros((8, 8))
    b = np.zeros(8)
    for i in range(4):
        x, y = s[i]
        u, v = d[i]
        A[2 * i] = [x, y, 1.0, 0.0, 0.0, 0.0, -u * x, -u * y]
        A[2 * i + 1] = [0.0, 0.0, 0.0, x, y, 1.0, -v * x, -v * y]
        b[2 * i], b[2 * i + 1] = u, v
    h = np.linalg.solve(A, b)
    return np.append(h, 1.0).reshape(3, 3)


def residuals(H, pa, pb):
    """|H(p_a) - p_b| per match; inf where w <= 0."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    w = H[2, 0] * pa[:, 0] + H[2, 1] * pa[:, 1] + H[2, 2]
    u = H[0, 0] * pa[:, 0] + H[0, 1] * pa[:, 1] + H[0, 2]
    v = H[1, 0] * pa[:, 0] + H[1, 1] * pa[:, 1] + H[1, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        ex, ey = u / w - pb[:, 0], v / w - pb[:, 1]
        r = np.sqrt(ex * ex + ey * ey)
    return np.where(w > 0, r, np.inf)


def normalizing_transform(p):
    """Hartley's normalisation: translate the centroid to 0 and scale the mean distance to
    sqrt(2); None if the points coincide."""
    p = np.asarray(p, np.float64)
    c = p.mean(axis=0)
    d = np.sqrt(((p - c) ** 2).sum(axis=1)).mean()
    if not d > 0:
        return None
    s = np.sqrt(2.0) / d
    return np.array([[s, 0.0, -s * c[0]], [0.0, s, -s * c[1]], [0.0, 0.0, 1.0]])


def refit_homography(pa, pb):
    """Least-squares homography (h33 = 1) over >= 4 correspondences in Hartley-normalised
    coordinates (numpy.linalg.lstsq), mapped back; None with fewer than 4 points or
    coincident points."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    if len(pa) < 4:
        return None
    Ta, Tb = normalizing_transform(pa), normalizing_transform(pb)
    if Ta is None or Tb is None:
        return None
    a = pa @ Ta[:2, :2].T + Ta[:2, 2]
    b = pb @ Tb[:2, :2].T + Tb[:2, 2]
    m = len(a)
    A = np.zeros((2 * m, 8))
    r = np.zeros(2 * m)
    A[0::2, 0], A[0::2, 1], A[0::2, 2] = a[:, 0], a[:, 1], 1.0
    A[0::2, 6], A[0::2, 7] = -b[:, 0] * a[:, 0], -b[:, 0] * a[:, 1]
    A[1::2, 3], A[1::2, 4], A[1::2, 5] = a[:, 0], a[:, 1], 1.0
    A[1::2, 6], A[1::2, 7] = -b[:, 1] * a[:, 0], -b[:, 1] * a[:, 1]
    r[0::2], r[1::2] = b[:, 0], b[:, 1]
    h = np.linalg.lstsq(A, r, rcond=None)[0]
    H = np.linalg.inv(Tb) @ np.append(h, 1.0).reshape(3, 3) @ Ta
    return H / H[2, 2]


def ransac(pa, pb, samples, th: float):
    """Score every sample; returns (scores [K], best index or -1, H of the best or None,
    inlier mask of the best [n] bool).  H is the least-squares refit over the best
    sample's inliers (refit_homography), or the sample's own H if that has no solution;
    the inlier mask is the best sample's."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    scores = np.full(len(samples), -1, np.int64)
    Hs = [None] * len(samples)
    for k, idx in enumerate(np.asarray(samples, np.int64)):
        H = homography_from_4(pa[idx], pb[idx])
        if H is None:
            continue
        Hs[k] = H
        scores[k] = int(np.sum(residuals(H, pa, pb) <= th))
    if len(samples) == 0 or scores.max() < 0:
        return scores, -1, None, np.zeros(len(pa), bool)
    best = int(np.argmax(scores))                # first maximum: lowest index on ties
    inl = residuals(Hs[best], pa, pb) <= th
    H = refit_homography(pa[inl], pb[inl])
    return scores, best, (Hs[best] if H is None else H), inl


def inlier_ratio(n_inliers: int, n_points: int) -> float:
    """Eq. (7): In_Num / Pt_Num (as a fraction; 0 for no points)."""
    return n_inliers / n_points if n_points > 0 else 0.0


def scaling_coefficient(pa, pb, des):
    """Eq. (1): f = sum_i (|a_i a_{i+1}| - |b_i b_{i+1}|) (1 - (Des(i) + Des(i+1)) / 1000) over
    consecutive matches i = 0 .. m-2 (in the order given), |.| the Euclidean segment length in
    pixels and Des the matches' descriptor distances.  f > 0: the segments are longer in image
    A, which is then the better base for simulation (Sec. III.A).  The printed summation bound
    is garbled; every consecutive pair is read as one segment."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    d = np.asarray(des, np.float64)
    if len(pa) < 2:
        return 0.0
    la = np.sqrt(((pa[1:] - pa[:-1]) ** 2).sum(axis=1))
    lb = np.sqrt(((pb[1:] - pb[:-1]) ** 2).sum(axis=1))
    w = 1.0 - (d[:-1] + d[1:]) / 1000.0
    return float(np.sum((la - lb) * w))
