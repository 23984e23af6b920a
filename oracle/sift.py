"""SIFT keypoints and 128-D descriptors (the detector and descriptor the paper uses for base-image
selection, Sec. III.A, and for precise matching on the re-simulated reference, Sec. III.C; the
method is that of Lowe [14]).

Test infrastructure only (see the package docstring).

The paper does not restate SIFT; each step below follows Lowe's construction [14], with the
readings a plain definition needs written out:

  * scale space: intensities as float32 0..255; the input is taken to carry a blur of
    sigma_in = 0.5 and is blurred to sigma0 = 1.6; each octave holds s + 3 Gaussian images
    G_k of blur sigma0 2^(k/s) (s = 3 layers), each made from the previous one by the
    incremental blur sqrt(sigma_k^2 - sigma_(k-1)^2); the next octave starts from every second
    pixel of G_s; octaves run while the image keeps at least 2^4 pixels on its short side
    (floor(log2 min(W, H)) - 3 octaves); no initial doubling of the image;
  * a Gaussian blur is separable, taps exp(-k^2 / (2 sigma^2)) for |k| <= ceil(4 sigma), summed
    and normalised in fp64 and rounded to float32; borders replicate the edge pixel; each pass
    sums w_k v_k in float32 from k = -r to r, every product and sum rounded (no fused
    multiply-add), rows first, then columns;
  * DoG images D_k = G_(k+1) - G_k in float32;
  * candidates: pixels of layers 1..s at least 5 pixels from the border with |D| above half
    the contrast threshold and strictly above (or strictly below) all 26 neighbours;
  * localisation: the quadratic fit of [14] (gradient and Hessian by central differences,
    in fp64 from the float32 D values), solved by cofactors: with n = -adj(H) g the offset is
    n / det(H); a sample is accepted when |n_i| < |det| / 2 for all three components, otherwise
    it moves one sample towards each component with |n_i| >= |det| / 2 (at most 5 fits; a
    move out of layers 1..s or the border region rejects it); all decisions are taken on
    products, without a division, so that any evaluation in the same operation order reaches
    the same ones;
  * rejection: |D(x^)| = |D det + g.n / 2| / |det| below 255 c / s (c = 0.04), or the 2x2
    spatial Hessian with det <= 0 or tr^2 r >= (r + 1)^2 det (r = 10);
  * orientation: a 36-bin histogram of the gradient directions atan2(dy, dx) (image axes, y
    down; bin = floor(36 angle / 2 pi + 1/2) mod 36) over the square of radius round(4.5 sigma)
    around the sample in the keypoint's Gaussian image, weighted by the gradient magnitude and a
    Gaussian of 1.5 sigma (sigma = the keypoint's blur in octave pixels); the histogram is
    smoothed circularly by (1, 4, 6, 4, 1) / 16; every local peak of at least 0.8 times the
    highest gives a keypoint, its angle refined by a parabola through the peak and its
    neighbours;
  * descriptor: 4 x 4 spatial cells of 3 sigma by 8 direction bins over a window rotated to the
    keypoint's angle, each sample's gradient magnitude weighted by a Gaussian of half the window
    (2 cells) and spread over the 8 neighbouring bins by trilinear interpolation; the 128 values
    are normalised to unit length, clipped at 0.2, renormalised, and stored as 8 bits:
    min(255, floor(512 v + 1/2));
  * order: keypoints in the order of their candidates (octave, candidate layer, row, column,
    before any move of the fit), the peaks of one candidate in bin order; the first
    max_keypoints are kept.

Parity status: pinned.  The tap table against the closed form of a sampled Gaussian; a blur of
a constant stays constant and a blurred impulse has the taps as its row and column profile;
DoG of a constant image has no candidate; candidates against a brute-force 26-neighbour loop;
the quadratic fit recovers the exact offset of a sampled quadratic; a Gaussian blob is found at
its centre with a scale near its own; orientation of a blob with a linear ramp follows the
ramp; a 90-degree rotation (an exact resampling) maps keypoints onto rotated keypoints, turns
orientations by pi / 2 and leaves descriptors unchanged; descriptors have the stated norm
and clip properties.
"""
from __future__ import annotations

import math

import numpy as np

N_LAYERS = 3
SIGMA0 = 1.6
SIGMA_IN = 0.5
CONTRAST = 0.04
EDGE = 10.0
BORDER = 5
MAX_FIT_STEPS = 5
ORI_BINS = 36
ORI_PEAK = 0.8
DESC_CELLS = 4
DESC_BINS = 8

KEYPOINT_DTYPE = np.dtype([("x", "f8"), ("y", "f8"), ("size", "f8"), ("angle", "f8"), ("response", "f8"),
                           ("octave", "i4"), ("layer", "i4"), ("xi", "i4"), ("yi", "i4"), ("peak", "i4"),
                           ("sigma_oct", "f8")])


def gaussian_taps(sigma: float) -> np.ndarray:
    """float32 taps w_k, k = -r..r, r = ceil(4 sigma): exp(-k^2 / (2 sigma^2)) / sum, in fp64."""
    r = int(math.ceil(4.0 * sigma))
    raw = [math.exp(-(k * k) / (2.0 * sigma * sigma)) for k in range(-r, r + 1)]
    total = 0.0
    for v in raw:
        total += v
    return np.array([v / total for v in raw], np.float64).astype(np.float32)


def blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of a float32 image: rows, then columns, each a float32 sum of
    rounded products from tap -r to tap r; edge pixels replicated."""
    w = gaussian_taps(sigma)
    r = (len(w) - 1) // 2
    a = np.asarray(img, np.float32)
    H, W = a.shape
    cols = np.clip(np.arange(W)[None, :] + np.arange(-r, r + 1)[:, None], 0, W - 1)
    acc = np.zeros_like(a)
    for i in range(2 * r + 1):
        acc = acc + w[i] * a[:, cols[i]]
    rows = np.clip(np.arange(H)[None, :] + np.arange(-r, r + 1)[:, None], 0, H - 1)
    out = np.zeros_like(acc)
    for i in range(2 * r + 1):
        out = out + w[i] * acc[rows[i], :]
    return out


def octave_count(W: int, H: int) -> int:
    return max(1, int(math.floor(math.log2(min(W, H)))) - 3)


def layer_sigmas(n_layers: int = N_LAYERS, sigma0: float = SIGMA0, sigma_in: float = SIGMA_IN):
    """Blur applied to make G_0 of the first octave, then the incremental blurs of G_1..G_(s+2)."""
    base = math.sqrt(sigma0 * sigma0 - sigma_in * sigma_in)
    inc = []
    for k in range(1, n_layers + 3):
        prev = sigma0 * math.pow(2.0, (k - 1) / n_layers)
        total = sigma0 * math.pow(2.0, k / n_layers)
        inc.append(math.sqrt(total * total - prev * prev))
    return base, inc


def gaussian_pyramid(img_u8, n_octaves: int = 0, n_layers: int = N_LAYERS, sigma0: float = SIGMA0,
                     sigma_in: float = SIGMA_IN):
    """[octave][k] float32 Gaussian images, k = 0 .. n_layers + 2."""
    a = np.asarray(img_u8, np.uint8).astype(np.float32)
    H, W = a.shape
    n_oct = n_octaves if n_octaves > 0 else octave_count(W, H)
    base, inc = layer_sigmas(n_layers, sigma0, sigma_in)
    pyr = []
    for o in range(n_oct):
        g0 = blur(a, base) if o == 0 else pyr[o - 1][n_layers][0::2, 0::2].copy()
        layers = [g0]
        for k in range(1, n_layers + 3):
            layers.append(blur(layers[-1], inc[k - 1]))
        pyr.append(layers)
    return pyr


def dog_pyramid(gauss):
    return [[(g[k + 1] - g[k]).astype(np.float32) for k in range(len(g) - 1)] for g in gauss]


def contrast_threshold(contrast: float = CONTRAST, n_layers: int = N_LAYERS) -> float:
    return contrast / n_layers * 255.0


def find_candidates(dog, n_layers: int = N_LAYERS, contrast: float = CONTRAST):
    """(octave, layer, y, x) of the 26-neighbour strict extrema above half the threshold,
    in (octave, layer, raster) order."""
    pre = 0.5 * contrast_threshold(contrast, n_layers)
    out = []
    for o, D in enumerate(dog):
        H, W = D[0].shape
        if H <= 2 * BORDER or W <= 2 * BORDER:
            continue
        for k in range(1, n_layers + 1):
            c = D[k][BORDER:H - BORDER, BORDER:W - BORDER]
            is_max = c > 0
            is_min = c < 0
            for dk in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if dk == 0 and dy == 0 and dx == 0:
                            continue
                        nb = D[k + dk][BORDER + dy:H - BORDER + dy, BORDER + dx:W - BORDER + dx]
                        is_max &= c > nb
                        is_min &= c < nb
            sel = (is_max | is_min) & (np.abs(c.astype(np.float64)) > pre)
            ys, xs = np.nonzero(sel)
            for y, x in zip(ys, xs):
                out.append((o, k, int(y) + BORDER, int(x) + BORDER))
    return out


def fit(D, k: int, y: int, x: int):
    """The quadratic fit at one sample, in fp64 from the float32 DoG values (in this operation
    order): (g, H entries, det, n = -adj(H) g)."""
    f = lambda kk, yy, xx: float(D[kk][yy, xx])
    c = f(k, y, x)
    g0 = (f(k, y, x + 1) - f(k, y, x - 1)) * 0.5
    g1 = (f(k, y + 1, x) - f(k, y - 1, x)) * 0.5
    g2 = (f(k + 1, y, x) - f(k - 1, y, x)) * 0.5
    v2 = c * 2.0
    dxx = (f(k, y, x + 1) + f(k, y, x - 1)) - v2
    dyy = (f(k, y + 1, x) + f(k, y - 1, x)) - v2
    dss = (f(k + 1, y, x) + f(k - 1, y, x)) - v2
    dxy = ((f(k, y + 1, x + 1) - f(k, y + 1, x - 1)) - (f(k, y - 1, x + 1) - f(k, y - 1, x - 1))) * 0.25
    dxs = ((f(k + 1, y, x + 1) - f(k + 1, y, x - 1)) - (f(k - 1, y, x + 1) - f(k - 1, y, x - 1))) * 0.25
    dys = ((f(k + 1, y + 1, x) - f(k + 1, y - 1, x)) - (f(k - 1, y + 1, x) - f(k - 1, y - 1, x))) * 0.25
    a00 = dyy * dss - dys * dys
    a01 = dxs * dys - dxy * dss
    a02 = dxy * dys - dyy * dxs
    a11 = dxx * dss - dxs * dxs
    a12 = dxy * dxs - dxx * dys
    a22 = dxx * dyy - dxy * dxy
    det = (dxx * a00 + dxy * a01) + dxs * a02
    n0 = -((a00 * g0 + a01 * g1) + a02 * g2)
    n1 = -((a01 * g0 + a11 * g1) + a12 * g2)
    n2 = -((a02 * g0 + a12 * g1) + a22 * g2)
    return dict(c=c, g=(g0, g1, g2), dxx=dxx, dyy=dyy, dxy=dxy, det=det, n=(n0, n1, n2))


def localise(D, o: int, k: int, y: int, x: int, n_layers: int = N_LAYERS, sigma0: float = SIGMA0,
             contrast: float = CONTRAST, edge: float = EDGE):
    """The accepted keypoint of candidate (o, k, y, x), or None."""
    H, W = D[0].shape
    conv = False
    F = None
    for _ in range(MAX_FIT_STEPS):
        F = fit(D, k, y, x)
        det = F["det"]
        if det == 0.0:
            return None
        half = 0.5 * abs(det)
        n = F["n"]
        if abs(n[0]) < half and abs(n[1]) < half and abs(n[2]) < half:
            conv = True
            break
        step = [0 if abs(v) < half else (1 if (v > 0.0) == (det > 0.0) else -1) for v in n]
        x += step[0]
        y += step[1]
        k += step[2]
        if k < 1 or k > n_layers or x < BORDER or x >= W - BORDER or y < BORDER or y >= H - BORDER:
            return None
    if not conv:
        return None
    det, n, g = F["det"], F["n"], F["g"]
    ad = abs(det)
    t = (g[0] * n[0] + g[1] * n[1]) + g[2] * n[2]
    lhs = abs(F["c"] * det + 0.5 * t)
    if lhs < contrast_threshold(contrast, n_layers) * ad:
        return None
    tr = F["dxx"] + F["dyy"]
    d2 = F["dxx"] * F["dyy"] - F["dxy"] * F["dxy"]
    if d2 <= 0.0 or tr * tr * edge >= (edge + 1.0) * (edge + 1.0) * d2:
        return None
    ox, oy, os_ = n[0] / det, n[1] / det, n[2] / det
    sigma_oct = sigma0 * math.pow(2.0, (k + os_) / n_layers)
    scale = float(1 << o)
    return dict(octave=o, layer=k, xi=x, yi=y, x=(x + ox) * scale, y=(y + oy) * scale,
                size=sigma_oct * scale, sigma_oct=sigma_oct, response=lhs / ad)


def _gradient(G, yy, xx):
    """Central differences (fp64, exact for float32 inputs) at integer points."""
    dx = G[yy, xx + 1].astype(np.float64) - G[yy, xx - 1].astype(np.float64)
    dy = G[yy + 1, xx].astype(np.float64) - G[yy - 1, xx].astype(np.float64)
    return dx, dy


def orientation_histogram(G, x: int, y: int, sigma_oct: float) -> np.ndarray:
    """The raw 36-bin histogram (fp64) around (x, y) of the float32 Gaussian image G."""
    H, W = G.shape
    R = int(math.floor(4.5 * sigma_oct + 0.5))
    sw = 1.5 * sigma_oct
    expf = -1.0 / (2.0 * sw * sw)
    i, j = np.mgrid[-R:R + 1, -R:R + 1]
    yy, xx = y + i, x + j
    ok = (yy > 0) & (yy < H - 1) & (xx > 0) & (xx < W - 1)
    i, j, yy, xx = i[ok], j[ok], yy[ok], xx[ok]
    dx, dy = _gradient(G, yy, xx)
    wgt = np.exp((i * i + j * j).astype(np.float64) * expf)
    mag = np.sqrt(dx * dx + dy * dy)
    ang = np.arctan2(dy, dx)
    b = np.floor(ang * (ORI_BINS / (2.0 * math.pi)) + 0.5).astype(np.int64) % ORI_BINS
    hist = np.zeros(ORI_BINS)
    np.add.at(hist, b, wgt * mag)
    return hist


def orientation_peaks(hist):
    """[(peak bin, angle in [0, 2 pi))] of the smoothed histogram, in bin order."""
    n = len(hist)
    h = np.asarray(hist, np.float64)
    s = np.array([(h[(i - 2) % n] + h[(i + 2) % n]) * (1.0 / 16.0) + (h[(i - 1) % n] + h[(i + 1) % n]) * (4.0 / 16.0)
                  + h[i] * (6.0 / 16.0) for i in range(n)])
    mx = s.max()
    out = []
    for i in range(n):
        l, c, r = s[(i - 1) % n], s[i], s[(i + 1) % n]
        if c > l and c > r and c >= ORI_PEAK * mx:
            bf = i + 0.5 * (l - r) / ((l - 2.0 * c) + r)
            if bf < 0.0:
                bf += n
            elif bf >= n:
                bf -= n
            ang = bf * (2.0 * math.pi / n)
            if ang >= 2.0 * math.pi:
                ang -= 2.0 * math.pi
            out.append((i, ang))
    return out


def descriptor(G, x: int, y: int, angle: float, sigma_oct: float) -> np.ndarray:
    """The 128 u8 values at (x, y) of the Gaussian image G for a keypoint of this angle."""
    H, W = G.shape
    d, nb = DESC_CELLS, DESC_BINS
    hw = 3.0 * sigma_oct
    radius = int(math.floor(hw * math.sqrt(2.0) * (d + 1) * 0.5 + 0.5))
    radius = min(radius, int(math.sqrt(float(W * W + H * H))))
    ct = math.cos(angle) / hw
    st = math.sin(angle) / hw
    bins_per_rad = nb / (2.0 * math.pi)
    expf = -1.0 / (0.5 * d * d)
    i, j = np.mgrid[-radius:radius + 1, -radius:radius + 1]
    i = i.astype(np.float64)
    j = j.astype(np.float64)
    # the offset (j, i) in the keypoint's frame: rotated by -angle (angle measured in image axes)
    c_rot = j * ct + i * st
    r_rot = i * ct - j * st
    rbin = r_rot + (d / 2 - 0.5)
    cbin = c_rot + (d / 2 - 0.5)
    yy = (y + i).astype(np.int64)
    xx = (x + j).astype(np.int64)
    ok = (rbin > -1) & (rbin < d) & (cbin > -1) & (cbin < d) & (yy > 0) & (yy < H - 1) & (xx > 0) & (xx < W - 1)
    c_rot, r_rot, rbin, cbin, yy, xx = c_rot[ok], r_rot[ok], rbin[ok], cbin[ok], yy[ok], xx[ok]
    dx, dy = _gradient(G, yy, xx)
    mag = np.sqrt(dx * dx + dy * dy)
    ang = np.arctan2(dy, dx)
    wgt = np.exp((c_rot * c_rot + r_rot * r_rot) * expf)
    ob = (ang - angle) * bins_per_rad
    ob = np.where(ob < 0, ob + nb, ob)
    ob = np.where(ob < 0, ob + nb, ob)
    ob = np.where(ob >= nb, ob - nb, ob)
    v = mag * wgt
    r0 = np.floor(rbin)
    c0 = np.floor(cbin)
    o0 = np.floor(ob)
    fr, fc, fo = rbin - r0, cbin - c0, ob - o0
    r0 = r0.astype(np.int64)
    c0 = c0.astype(np.int64)
    o0 = o0.astype(np.int64) % nb
    hist = np.zeros((d + 2, d + 2, nb))
    for dr, wr in ((0, 1.0 - fr), (1, fr)):
        for dc, wc in ((0, 1.0 - fc), (1, fc)):
            for do, wo in ((0, 1.0 - fo), (1, fo)):
                np.add.at(hist, (r0 + 1 + dr, c0 + 1 + dc, (o0 + do) % nb), v * wr * wc * wo)
    desc = hist[1:d + 1, 1:d + 1, :].reshape(-1)
    nrm = math.sqrt(float(np.sum(desc * desc)))
    desc = np.minimum(desc, 0.2 * nrm)
    nrm2 = math.sqrt(float(np.sum(desc * desc)))
    scale = 512.0 / max(nrm2, 1.1920928955078125e-07)
    return np.minimum(np.floor(desc * scale + 0.5), 255.0).astype(np.uint8)


def extract(img_u8, max_keypoints: int = 4096, n_octaves: int = 0, n_layers: int = N_LAYERS,
            sigma0: float = SIGMA0, sigma_in: float = SIGMA_IN, contrast: float = CONTRAST, edge: float = EDGE):
    """(keypoints [KEYPOINT_DTYPE], descriptors u8 [n, 128], total found) of an 8-bit image."""
    gauss = gaussian_pyramid(img_u8, n_octaves, n_layers, sigma0, sigma_in)
    dog = dog_pyramid(gauss)
    kps = []
    for (o, k, y, x) in find_candidates(dog, n_layers, contrast):
        loc = localise(dog[o], o, k, y, x, n_layers, sigma0, contrast, edge)
        if loc is None:
            continue
        G = gauss[o][loc["layer"]]
        hist = orientation_histogram(G, loc["xi"], loc["yi"], loc["sigma_oct"])
        for peak, ang in orientation_peaks(hist):
            kp = dict(loc)
            kp["peak"] = peak
            kp["angle"] = ang
            kps.append(kp)
    total = len(kps)
    kps = kps[:max_keypoints]
    out = np.zeros(len(kps), KEYPOINT_DTYPE)
    desc = np.zeros((len(kps), DESC_CELLS * DESC_CELLS * DESC_BINS), np.uint8)
    for i, kp in enumerate(kps):
        for f in KEYPOINT_DTYPE.names:
            out[i][f] = kp[f]
        desc[i] = descriptor(gauss[kp["octave"]][kp["layer"]], kp["xi"], kp["yi"], kp["angle"], kp["sigma_oct"])
    return out, desc, total
