"""ORB on one simulated view: pyramid, FAST-9, Harris top-N, orientation, smoothing, rBRIEF-256.

Test infrastructure only (see the package docstring).  Everything here is exact
integer arithmetic on u8 images, so the GPU must reproduce it bit for bit.

The paper uses ORB (oFAST + rBRIEF, Sec. V.A) with 1000 points per image
(Sec. IV.C) to score every simulated view; ORB's internals are not restated in
the paper, so each step below follows the ORB construction, made exact:
  * pyramid: levels at factor 1.2, fixed-point bilinear (weights in 1/2048),
    each level built from the previous one;
  * FAST-9 with threshold T: corner iff some arc of 9 contiguous pixels of the
    16-pixel radius-3 circle is brighter than I_p + T or darker than I_p - T;
    the score V is the largest threshold a pixel still passes at (max over
    arcs and polarities of the arc minimum of the signed differences);
    3x3 non-maximum suppression with ties broken by raster order;
  * Harris response at each surviving corner, integer form 25 det - tr^2 of
    the 7x7 structure tensor of 3x3 Sobel gradients; per-level top n_l;
  * orientation from the intensity centroid over a radius-15 disk, quantised
    to 30 bins of 12 deg by an integer argmax;
  * rBRIEF: 256 tests of a given point-pair pattern, rotated to the bin, on a
    7-tap integer Gaussian smoothing of the level.

Parity status: pinned (brute-force FAST on small images, closed-form Harris
cases and agreement with a scipy Sobel / box-filter Harris, ramp-patch
orientations, scipy correlate for the smoothing, 180-degree rotation
equivariance of orientation and descriptors).
"""
from __future__ import annotations

import math

import numpy as np

BORDER = 22            # detection border: BRIEF tests reach 21 px after rotation
HARRIS_HALF = 3        # 7x7 window
ORIENT_RADIUS = 15
N_BINS = 30
SMOOTH_TAPS = np.array([18, 34, 49, 54, 49, 34, 18], np.int64)   # sums to 256

# Bresenham circle of radius 3, clockwise from 12 o'clock (x right, y down).
CIRCLE = np.array([(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
                   (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)], np.int64)
ARC = 9


# ---------------------------------------------------------------------------- pyramid

def _resample_index(n_dst: int, n_src: int):
    """Fixed-point source position of each destination index for a bilinear
    down-scale from n_src to n_dst samples.

    src = (d + 1/2) n_src / n_dst - 1/2 in units of 1/2048, rounded half up,
    computed exactly in integers: 2048 * src = 1024 ((2d+1) n_src - n_dst) / n_dst.
    Returns (i0, i1, w0, w1) with w0 + w1 = 2048."""
    d = np.arange(n_dst, dtype=np.int64)
    num = 1024 * ((2 * d + 1) * n_src - n_dst)
    q = (2 * num + n_dst) // (2 * n_dst)          # round half up (num >= 0)
    i0 = q >> 11
    w1 = q & 2047
    over = i0 >= n_src - 1
    i0 = np.where(over, n_src - 1, i0)
    w1 = np.where(over, 0, w1)
    i1 = np.minimum(i0 + 1, n_src - 1)
    return i0, i1, 2048 - w1, w1


def pyr_down(img_u8, mask, dst_w: int, dst_h: int):
    """One pyramid step: out = (sum_{2x2} wy wx pix + 2^21) >> 22 with 11-bit weights;
    a level pixel holds content iff all four source pixels of its footprint do."""
    P = np.asarray(img_u8, np.int64)
    Mk = np.asarray(mask, bool)
    H, W = P.shape
    x0, x1, wx0, wx1 = _resample_index(dst_w, W)
    y0, y1, wy0, wy1 = _resample_index(dst_h, H)
    top = wx0[None, :] * P[y0][:, x0] + wx1[None, :] * P[y0][:, x1]
    bot = wx0[None, :] * P[y1][:, x0] + wx1[None, :] * P[y1][:, x1]
    out = (wy0[:, None] * top + wy1[:, None] * bot + (1 << 21)) >> 22
    mo = Mk[y0][:, x0] & Mk[y0][:, x1] & Mk[y1][:, x0] & Mk[y1][:, x1]
    return out.astype(np.uint8), mo


def build_pyramid(view_u8, mask, dims):
    """Levels 0..L-1; level 0 is the view itself, dims[l] = (W_l, H_l)."""
    levels = [(np.asarray(view_u8, np.uint8), np.asarray(mask, bool))]
    for (w, h) in dims[1:]:
        levels.append(pyr_down(levels[-1][0], levels[-1][1], w, h))
    return levels


# ---------------------------------------------------------------------------- FAST-9

def fast_score(P):
    """FAST-9 score V on the pixels whose circle lies inside the image.

    Returns V (int64, H x W) with V = -10**6 where the circle does not fit.
    V(p) = max over the 16 arcs of 9 contiguous circle pixels, and over the two
    polarities, of the minimum over the arc of (I_c - I_p) (bright) or
    (I_p - I_c) (dark).  p is a corner at threshold T iff V(p) > T."""
    I = np.asarray(P, np.int64)
    H, W = I.shape
    V = np.full((H, W), -10 ** 6, np.int64)
    if H < 7 or W < 7:
        return V
    c = I[3:H - 3, 3:W - 3]
    d = np.stack([I[3 + dy:H - 3 + dy, 3 + dx:W - 3 + dx] - c for dx, dy in CIRCLE])   # (16, h, w)
    best = np.full(c.shape, -10 ** 6, np.int64)
    for s in range(16):
        arc = d[[(s + j) % 16 for j in range(ARC)]]
        best = np.maximum(best, arc.min(axis=0))          # bright arc starting at s
        best = np.maximum(best, (-arc).min(axis=0))       # dark arc starting at s
    V[3:H - 3, 3:W - 3] = best
    return V


def fast_candidates(P, mask, threshold: int, border: int = BORDER):
    """FAST corners that survive non-maximum suppression and the content filter.

    * corner(p)  <=> V(p) > threshold
    * p is kept iff it is a corner inside [border, W-border) x [border, H-border),
      every corner q among its 8 neighbours has V(q) < V(p), or V(q) == V(p)
      and q comes after p in raster order,
    * and the four corners of the box p +- border hold image content
      (mask == 1), so the patch used by Harris, orientation and BRIEF never
      touches the zero fill outside the simulated view.
    Returns (xs, ys) int64 arrays in raster order."""
    P = np.asarray(P)
    Mk = np.asarray(mask, bool)
    H, W = P.shape
    if W <= 2 * border or H <= 2 * border:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    V = fast_score(P)
    corner = V > threshold
    ys, xs = np.nonzero(corner)
    keep = (xs >= border) & (xs < W - border) & (ys >= border) & (ys < H - border)
    xs, ys = xs[keep], ys[keep]
    ok = np.ones(xs.size, bool)
    vp = V[ys, xs]
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            qx, qy = xs + dx, ys + dy
            vq = V[qy, qx]
            cq = corner[qy, qx]
            q_after = (dy > 0) or (dy == 0 and dx > 0)
            wins = (vp > vq) | ((vp == vq) & q_after)
            ok &= (~cq) | wins
    b = border
    ok &= Mk[ys - b, xs - b] & Mk[ys - b, xs + b] & Mk[ys + b, xs - b] & Mk[ys + b, xs + b]
    return xs[ok], ys[ok]


# ---------------------------------------------------------------------------- Harris

def harris_response(P, xs, ys):
    """R = 25 (a b - c^2) - (a + b)^2 (= 25 (det - 0.04 tr^2)) in int64, where
    a = sum Ix^2, b = sum Iy^2, c = sum Ix Iy over the 7x7 window centred on p and
    Ix, Iy are 3x3 Sobel derivatives (x to the right, y downwards)."""
    I = np.asarray(P, np.int64)
    xs = np.asarray(xs, np.int64)
    ys = np.asarray(ys, np.int64)
    r = HARRIS_HALF + 1
    off = np.arange(-r, r + 1)
    patch = I[(ys[:, None, None] + off[None, :, None]), (xs[:, None, None] + off[None, None, :])]  # (n, 9, 9)
    # Sobel on the inner 7x7
    p = patch
    ix = (p[:, :-2, 2:] + 2 * p[:, 1:-1, 2:] + p[:, 2:, 2:]) - (p[:, :-2, :-2] + 2 * p[:, 1:-1, :-2] + p[:, 2:, :-2])
    iy = (p[:, 2:, :-2] + 2 * p[:, 2:, 1:-1] + p[:, 2:, 2:]) - (p[:, :-2, :-2] + 2 * p[:, :-2, 1:-1] + p[:, :-2, 2:])
    a = (ix * ix).sum(axis=(1, 2))
    b = (iy * iy).sum(axis=(1, 2))
    c = (ix * iy).sum(axis=(1, 2))
    return 25 * (a * b - c * c) - (a + b) * (a + b)


def select_top(R, raster, quota: int):
    """Indices of the top `quota` entries by (R descending, raster ascending), in that order."""
    order = np.lexsort((raster, -np.asarray(R, np.int64)))
    return order[:quota]


# ---------------------------------------------------------------------------- orientation

def orientation_table():
    """Integer unit vectors of the 30 bins: C_k = round(2^20 cos(2 pi k / 30)),
    S_k = round(2^20 sin(2 pi k / 30)) for k < 15 and the negatives for k + 15,
    so opposite bins are exact negatives of each other."""
    C = np.zeros(N_BINS, np.int64)
    S = np.zeros(N_BINS, np.int64)
    half = N_BINS // 2
    for k in range(half):
        a = 2.0 * math.pi * k / N_BINS
        C[k] = int(np.rint(math.cos(a) * (1 << 20)))
        S[k] = int(np.rint(math.sin(a) * (1 << 20)))
        C[k + half] = -C[k]
        S[k + half] = -S[k]
    return C, S


def disk_offsets(radius: int = ORIENT_RADIUS):
    ys, xs = np.mgrid[-radius:radius + 1, -radius:radius + 1]
    sel = xs * xs + ys * ys <= radius * radius
    return xs[sel].astype(np.int64), ys[sel].astype(np.int64)


def orientation_bins(P, xs, ys):
    """Intensity-centroid orientation: m10 = sum x I, m01 = sum y I over the disk of
    radius 15 (unsmoothed level image); bin = argmax_k (m10 C_k + m01 S_k),
    smallest k on ties (all-zero moments give bin 0)."""
    I = np.asarray(P, np.int64)
    dx, dy = disk_offsets()
    vals = I[np.asarray(ys)[:, None] + dy[None, :], np.asarray(xs)[:, None] + dx[None, :]]
    m10 = (vals * dx[None, :]).sum(axis=1)
    m01 = (vals * dy[None, :]).sum(axis=1)
    C, S = orientation_table()
    score = m10[:, None] * C[None, :] + m01[:, None] * S[None, :]
    return np.argmax(score, axis=1).astype(np.int64)


# ---------------------------------------------------------------------------- smoothing + rBRIEF

def smooth(P):
    """Separable 7-tap integer Gaussian [18 34 49 54 49 34 18] / 256 per axis,
    border replicated; horizontal sums are kept exact, the vertical pass rounds:
    S = (sum_j w_j h_j + 2^15) >> 16."""
    I = np.asarray(P, np.int64)
    H, W = I.shape
    xs = np.arange(W)
    ys = np.arange(H)
    h = np.zeros((H, W), np.int64)
    for k, w in enumerate(SMOOTH_TAPS):
        h += w * I[:, np.clip(xs + k - 3, 0, W - 1)]
    v = np.zeros((H, W), np.int64)
    for k, w in enumerate(SMOOTH_TAPS):
        v += w * h[np.clip(ys + k - 3, 0, H - 1), :]
    return ((v + (1 << 15)) >> 16).astype(np.uint8)


def _round_shift20(v):
    """sign(v) * ((|v| + 2^19) >> 20): rounds half away from zero, odd-symmetric."""
    v = np.asarray(v, np.int64)
    return np.sign(v) * ((np.abs(v) + (1 << 19)) >> 20)


def steer_pattern(pattern, b: int):
    """Rotate the test pattern (256 x (x1, y1, x2, y2)) to orientation bin b:
    (x, y) -> (rnd(x C_b - y S_b), rnd(x S_b + y C_b))."""
    C, S = orientation_table()
    pt = np.asarray(pattern, np.int64)
    out = np.empty_like(pt)
    for j in (0, 2):
        x, y = pt[:, j], pt[:, j + 1]
        out[:, j] = _round_shift20(x * C[b] - y * S[b])
        out[:, j + 1] = _round_shift20(x * S[b] + y * C[b])
    return out


def brief_descriptors(Sm, xs, ys, bins, pattern):
    """bit_i = [Sm(p + a_i') < Sm(p + b_i')] for the 256 steered tests; bit i is
    stored in byte i // 8 at bit position i % 8 (least significant first)."""
    Sm = np.asarray(Sm, np.int64)
    n = len(xs)
    out = np.zeros((n, 32), np.uint8)
    steered = {}
    for i in range(n):
        b = int(bins[i])
        if b not in steered:
            steered[b] = steer_pattern(pattern, b)
        st = steered[b]
        x, y = int(xs[i]), int(ys[i])
        va = Sm[y + st[:, 1], x + st[:, 0]]
        vb = Sm[y + st[:, 3], x + st[:, 2]]
        bits = (va < vb).astype(np.uint8)
        out[i] = np.packbits(bits, bitorder="little")
    return out


# ---------------------------------------------------------------------------- one view

def extract_view(view_u8, mask, dims, quotas, threshold: int, pattern, border: int = BORDER):
    """ORB on one view.  Keypoints come in canonical order: level ascending,
    then Harris response descending, then raster position ascending.

    Returns dict of arrays: x, y (level pixel coords), level, bin, harris,
    desc (n x 32 u8)."""
    levels = build_pyramid(view_u8, mask, dims)
    X, Y, LV, BN, RR, D = [], [], [], [], [], []
    for l, ((P, Mk), quota) in enumerate(zip(levels, quotas)):
        xs, ys = fast_candidates(P, Mk, threshold, border)
        if xs.size == 0 or quota <= 0:
            continue
        R = harris_response(P, xs, ys)
        raster = ys * P.shape[1] + xs
        sel = select_top(R, raster, quota)
        xs, ys, R = xs[sel], ys[sel], R[sel]
        bins = orientation_bins(P, xs, ys)
        Sm = smooth(P)
        D.append(brief_descriptors(Sm, xs, ys, bins, pattern))
        X.append(xs); Y.append(ys); LV.append(np.full(xs.size, l, np.int64)); BN.append(bins); RR.append(R)
    if not X:
        z = np.zeros(0, np.int64)
        return dict(x=z, y=z, level=z, bin=z, harris=z, desc=np.zeros((0, 32), np.uint8))
    return dict(x=np.concatenate(X), y=np.concatenate(Y), level=np.concatenate(LV),
                bin=np.concatenate(BN), harris=np.concatenate(RR), desc=np.concatenate(D))
