"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side tests.

This module renders test scenes and draws the random numbers the method needs
(the rBRIEF test pattern).  It contains none of the method's arithmetic: no
view-sampling rule, no anti-alias blur, no Lanczos resampling, no ORB step and
no matching.  Scenes are described in continuous coordinates and rendered by
point sampling with box supersampling, so that an image pair with a known
affine relation can be produced without running the method under test.

Scene recipe (a stand-in for the paper's Mikolajczyk / MorelYu image pairs,
which are not available): background 128, additive isotropic Gaussian blobs
(sigma ~ U[2, 12] px, amplitude ~ U[-96, 96]), then axis-aligned rectangles of
uniform random gray painted in order (later ones overwrite earlier ones), then
i.i.d. Gaussian noise with standard deviation 2 (variance 4), rounded and
clipped to 0..255.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "make_scene", "render", "affine_canvas", "tilt_rotation",
    "brief_pattern", "PairCase", "make_pair", "PAIR_CONFIGS", "rng", "make_crops", "crop_params",
    "batch_pairs",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for a given seed (all inputs are drawn from this)."""
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Scene:
    """A planar scene in continuous coordinates (pixel centres of the
    undistorted image at integer positions, the image covering
    [-0.5, W-0.5] x [-0.5, H-0.5])."""
    width: int
    height: int
    blobs: np.ndarray          # (nb, 4): cx, cy, sigma, amplitude
    rects: np.ndarray          # (nr, 5): x0, y0, x1, y1, gray  (half-open box)
    background: float = 128.0


def make_scene(width: int, height: int, n_blobs: int, n_rects: int, seed: int) -> Scene:
    g = rng(seed)
    bl = np.empty((n_blobs, 4), np.float64)
    bl[:, 0] = g.uniform(-0.5, width - 0.5, n_blobs)
    bl[:, 1] = g.uniform(-0.5, height - 0.5, n_blobs)
    bl[:, 2] = g.uniform(2.0, 12.0, n_blobs)
    bl[:, 3] = g.uniform(-96.0, 96.0, n_blobs)
    side_max = max(4, int(math.floor(0.15 * min(width, height))))
    rc = np.empty((n_rects, 5), np.float64)
    for i in range(n_rects):
        w = int(g.integers(4, side_max + 1))
        h = int(g.integers(4, side_max + 1))
        x0 = int(g.integers(0, max(1, width - w + 1)))
        y0 = int(g.integers(0, max(1, height - h + 1)))
        # the rectangle covers whole pixels x0..x0+w-1 of the undistorted image
        rc[i] = (x0 - 0.5, y0 - 0.5, x0 + w - 0.5, y0 + h - 0.5, float(g.integers(0, 256)))
    return Scene(width, height, bl, rc)


def tilt_rotation(t: float, phi: float, psi: float) -> np.ndarray:
    """Linear part of a camera change: rotate by phi, compress x by t, rotate by psi."""
    def rot(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, -s], [s, c]])
    return rot(psi) @ np.diag([1.0 / t, 1.0]) @ rot(phi)


def affine_canvas(M: np.ndarray, width: int, height: int):
    """Bounding canvas of the image of [-0.5,W-0.5]x[-0.5,H-0.5] under x -> M x.

    Returns (out_w, out_h, offset) with the image placed so that its bounding
    box starts at -0.5 in the output pixel grid: q = M p + offset."""
    cs = np.array([[-0.5, -0.5], [width - 0.5, -0.5], [-0.5, height - 0.5], [width - 0.5, height - 0.5]]).T
    mc = M @ cs
    lo, hi = mc.min(axis=1), mc.max(axis=1)
    ow = int(math.ceil(hi[0] - lo[0] - 1e-7))
    oh = int(math.ceil(hi[1] - lo[1] - 1e-7))
    return ow, oh, -lo - 0.5


def render(scene: Scene, M: np.ndarray, offset: np.ndarray, out_w: int, out_h: int,
           noise_seed: int, supersample: int = 4, noise_sigma: float = 2.0,
           quantize: bool = True, strip: int = 64) -> np.ndarray:
    """Render the scene seen through q = M p + offset (p scene coords, q output pixel coords).

    Each output pixel is the mean of supersample^2 point samples placed on a
    regular grid inside the pixel; each point sample is background + blobs,
    overwritten by the last rectangle that contains it."""
    M = np.asarray(M, np.float64)
    Minv = np.linalg.inv(M)
    off = np.asarray(offset, np.float64)
    k = supersample
    out = np.empty((out_h, out_w), np.float64)
    blobs, rects = scene.blobs, scene.rects

    def out_box(x0, y0, x1, y1):
        # bounding box, in output pixel coordinates, of a scene-space box
        cs = np.array([[x0, x1, x0, x1], [y0, y0, y1, y1]], np.float64)
        q = M @ cs + off[:, None]
        return q[0].min(), q[1].min(), q[0].max(), q[1].max()

    def to_index(lo, hi, n):
        # supersample index i sits at output coordinate -0.5 + (i + 0.5) / k
        a = max(0, int(math.ceil((lo + 0.5) * k - 0.5)))
        b = min(n - 1, int(math.floor((hi + 0.5) * k - 0.5)))
        return a, b + 1

    blob_boxes = [out_box(cx - 4 * sg, cy - 4 * sg, cx + 4 * sg, cy + 4 * sg) for cx, cy, sg, _ in blobs]
    rect_boxes = [out_box(r[0], r[1], r[2], r[3]) for r in rects]
    nxs = out_w * k
    qx_all = -0.5 + (np.arange(nxs) + 0.5) / k
    for y0 in range(0, out_h, strip):
        y1 = min(out_h, y0 + strip)
        r0, r1 = y0 * k, y1 * k
        qy = -0.5 + (np.arange(r0, r1) + 0.5) / k
        val = np.full((r1 - r0, nxs), scene.background)

        def window(box):
            ya, yb = to_index(box[1], box[3], out_h * k)
            ya, yb = max(ya, r0), min(yb, r1)
            xa, xb = to_index(box[0], box[2], nxs)
            if ya >= yb or xa >= xb:
                return None
            QX, QY = np.meshgrid(qx_all[xa:xb] - off[0], qy[ya - r0:yb - r0] - off[1])
            px = Minv[0, 0] * QX + Minv[0, 1] * QY
            py = Minv[1, 0] * QX + Minv[1, 1] * QY
            return (slice(ya - r0, yb - r0), slice(xa, xb)), px, py

        for (cx, cy, sg, amp), box in zip(blobs, blob_boxes):
            w = window(box)
            if w is None:
                continue
            sl, px, py = w
            dx = px - cx
            dy = py - cy
            val[sl] += amp * np.exp(-(dx * dx + dy * dy) / (2.0 * sg * sg))
        for (rx0, ry0, rx1, ry1, gray), box in zip(rects, rect_boxes):
            w = window(box)
            if w is None:
                continue
            sl, px, py = w
            inside = (px >= rx0) & (px < rx1) & (py >= ry0) & (py < ry1)
            sub = val[sl]
            sub[inside] = gray
        out[y0:y1] = val.reshape(y1 - y0, k, out_w, k).mean(axis=(1, 3))
    g = rng(noise_seed)
    if noise_sigma > 0:
        out = out + g.normal(0.0, noise_sigma, out.shape)
    if not quantize:
        return out
    return np.clip(np.rint(out), 0, 255).astype(np.uint8)


def brief_pattern(seed: int = 2011) -> np.ndarray:
    """256 binary-test point pairs (x1, y1, x2, y2), int8, each coordinate in [-15, 15].

    Drawn i.i.d. from an isotropic Gaussian of standard deviation 31/5 (the
    BRIEF sampling strategy for a 31x31 patch), rounded, clipped to +-15;
    pairs whose two points coincide are redrawn.  The learned test table of
    the ORB paper is not available, so this seeded draw stands in for it."""
    g = rng(seed)
    out = np.empty((256, 4), np.int8)
    i = 0
    while i < 256:
        v = np.clip(np.rint(g.normal(0.0, 31.0 / 5.0, 4)), -15, 15).astype(np.int64)
        if v[0] == v[2] and v[1] == v[3]:
            continue
        out[i] = v
        i += 1
    return out


@dataclass
class PairCase:
    """An image pair with a known map from image-A pixel coordinates to image-B pixel coordinates."""
    name: str
    A: np.ndarray
    B: np.ndarray
    H: np.ndarray              # 3x3, pB ~ H @ [pA, 1]
    meta: dict = field(default_factory=dict)


def make_pair(width: int, height: int, n_blobs: int, n_rects: int, seed: int,
              t: float, phi: float, psi: float, supersample: int = 4, name: str = "pair",
              t_a: float = 1.0, phi_a: float = 0.0) -> PairCase:
    """A = the scene seen head-on, or after a tilt t_a along longitude phi_a when t_a > 1;
    B = the scene after a tilt t along longitude phi and a rotation psi.  Each image covers the
    bounding box of the transformed scene."""
    sc = make_scene(width, height, n_blobs, n_rects, seed)
    if t_a == 1.0:
        MA, offa = np.eye(2), np.zeros(2)
        A = render(sc, MA, offa, width, height, noise_seed=seed * 7919 + 1, supersample=supersample)
    else:
        MA = tilt_rotation(t_a, phi_a, 0.0)
        aw, ah, offa = affine_canvas(MA, width, height)
        A = render(sc, MA, offa, aw, ah, noise_seed=seed * 7919 + 1, supersample=supersample)
    M = tilt_rotation(t, phi, psi)
    bw, bh, off = affine_canvas(M, width, height)
    B = render(sc, M, off, bw, bh, noise_seed=seed * 7919 + 2, supersample=supersample)
    # pB = M pS + off and pA = MA pS + offa  =>  pB = M MA^-1 (pA - offa) + off
    L = M @ np.linalg.inv(MA)
    H = np.eye(3)
    H[:2, :2] = L
    H[:2, 2] = off - L @ offa
    return PairCase(name, A, B, H, dict(t=t, phi=phi, psi=psi, seed=seed, t_a=t_a, phi_a=phi_a))


# Workload definitions (image sizes, scene density, ground-truth camera change).
PAIR_CONFIGS = {
    # 256x256, 40 blobs, 30 rectangles; B: tilt 2, rotation 30 deg.
    "tiny": dict(width=256, height=256, n_blobs=40, n_rects=30, seed=1, t=2.0, phi=0.0, psi=math.radians(30.0)),
    # 1024x768, 400 blobs, 300 rectangles; B: absolute tilt 4 (~75.5 deg), rotation 45 deg.
    "full": dict(width=1024, height=768, n_blobs=400, n_rects=300, seed=2, t=4.0, phi=0.0, psi=math.radians(45.0)),
    # 4096x3072, 4000 blobs, 3000 rectangles; A and B: absolute tilt 80 deg (t = 1 / cos 80 deg =
    # 5.76), A compressed along x, B along y (tilt along longitude 90 deg, turned back by -90 deg),
    # so the transition tilt from A to B is t^2 = 33.2 (88.3 deg).
    "stress": dict(width=4096, height=3072, n_blobs=4000, n_rects=3000, seed=4,
                   t_a=1.0 / math.cos(math.radians(80.0)), phi_a=0.0,
                   t=1.0 / math.cos(math.radians(80.0)), phi=math.radians(90.0), psi=math.radians(-90.0)),
}


def make_crops(n: int, size: int, seed: int, distinct: int = 0, supersample: int = 4) -> np.ndarray:
    """n fp32 crops of size x size with values in [0, 1] (the scene generator, u8 / 255).

    Scene density scales with area (133 blobs and 100 rectangles at 512 x 512).
    distinct > 0 renders only that many scenes and repeats them (for timing runs,
    where the content does not change the work)."""
    m = n if distinct <= 0 else min(distinct, n)
    area = size * size / (512.0 * 512.0)
    nb, nr = max(4, int(round(133 * area))), max(3, int(round(100 * area)))
    out = np.empty((n, size, size), np.float32)
    for i in range(m):
        sc = make_scene(size, size, nb, nr, seed + i)
        out[i] = render(sc, np.eye(2), np.zeros(2), size, size, noise_seed=(seed + i) * 7919 + 3,
                        supersample=supersample).astype(np.float32) / 255.0
    for i in range(m, n):
        out[i] = out[i % m]
    return out


def crop_params(n: int, seed: int, max_shift: float = 16.0) -> np.ndarray:
    """Camera parameters per crop, [n, 6] fp64 (t, phi, psi, s, tx, ty): t ~ U[1, 6],
    phi ~ U[0, pi), psi ~ U[-pi, pi), s ~ U[0.5, 1], tx, ty ~ U[-max_shift, max_shift]."""
    g = rng(seed)
    P = np.empty((n, 6))
    P[:, 0] = g.uniform(1.0, 6.0, n)
    P[:, 1] = g.uniform(0.0, math.pi, n)
    P[:, 2] = g.uniform(-math.pi, math.pi, n)
    P[:, 3] = g.uniform(0.5, 1.0, n)
    P[:, 4] = g.uniform(-max_shift, max_shift, n)
    P[:, 5] = g.uniform(-max_shift, max_shift, n)
    return P


def batch_pairs(n: int, seed: int = 3000, side_min: int = 480, side_max: int = 2048, supersample: int = 1):
    """n pairs of uneven sizes: width ~ U{side_min..side_max}, aspect ~ U[0.6, 1.6],
    height = clip(round(width / aspect), side_min, side_max); scene density scaled by
    area from 400 blobs / 300 rectangles at 1024 x 768; B = the scene under an absolute
    tilt ~ U[0, 80] degrees (t = 1 / cos), longitude ~ U[0, pi) and rotation ~ U[0, 2 pi).
    Pair k uses seed + k."""
    out = []
    for k in range(n):
        g = rng(seed + k)
        w = int(g.integers(side_min, side_max + 1))
        aspect = float(g.uniform(0.6, 1.6))
        h = int(np.clip(round(w / aspect), side_min, side_max))
        theta = math.radians(float(g.uniform(0.0, 80.0)))
        phi = float(g.uniform(0.0, math.pi))
        psi = float(g.uniform(0.0, 2.0 * math.pi))
        area = w * h / (1024.0 * 768.0)
        out.append(make_pair(w, h, max(8, int(round(400 * area))), max(6, int(round(300 * area))), seed + k,
                             1.0 / math.cos(theta), phi, psi, supersample=supersample, name=f"batch{k}"))
    return out


def sift_like_descriptors(n: int, seed: int) -> np.ndarray:
    """n x 128 u8 descriptors distributed like 8-bit SIFT descriptors: 128 gamma(0.6) magnitudes
    normalised to unit length, clipped at 0.2, renormalised, scaled by 512, rounded and clipped to
    0..255 (the usual quantisation of the SIFT descriptor)."""
    g = rng(seed)
    v = g.gamma(0.6, 1.0, (n, 128))
    v /= np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-12)
    v = np.minimum(v, 0.2)
    v /= np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-12)
    return np.clip(np.rint(v * 512.0), 0, 255).astype(np.uint8)


def sift_like_sets(n_q: int, n_t: int, seed: int, shared: float = 0.5, noise: float = 6.0):
    """Query and train sets of SIFT-like descriptors where a fraction `shared` of the queries are
    noisy copies (Gaussian noise of the given std, rounded, clipped) of random train descriptors,
    the rest independent, so that nearest-neighbour matching finds true pairs among distractors.
    Returns (queries, train, source) with source[q] = the train index copied, or -1."""
    g = rng(seed + 1)
    T = sift_like_descriptors(n_t, seed)
    Q = sift_like_descriptors(n_q, seed + 2)
    src = np.full(n_q, -1, np.int64)
    if n_t > 0:
        k = g.random(n_q) < shared
        src[k] = g.integers(0, n_t, int(k.sum()))
        Q[k] = np.clip(np.rint(T[src[k]].astype(np.float64) + g.normal(0.0, noise, (int(k.sum()), 128))), 0, 255)
    return np.ascontiguousarray(Q, np.uint8), np.ascontiguousarray(T, np.uint8), src
