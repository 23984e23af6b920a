"""Affine view simulation: directional anti-alias blur, Lanczos-4 resampling, quantisation.

Test infrastructure only (see the package docstring).

Parity status: pinned.  Nearest-neighbour sampling: the identity view and integer
translations reproduce the input, half-pixel positions round up, quarter turns equal
np.rot90.  Blur: axis-aligned cases equal scipy.ndimage.convolve1d
(mode 'nearest'), constants and ramps are preserved, and the impulse response
has its variance along the tilt direction.  Warp: closed forms of the kernel
of eq. (4), identity view reproduces the input, quarter turns equal np.rot90,
constants are preserved, band-limited images are reproduced at the mapped
points, and a scalar brute-force loop agrees on a small image.
"""
from __future__ import annotations

import math

import numpy as np

from .plan import View

LANCZOS_A = 4          # Sec. IV.C: n = 4, an 8x8 neighbourhood


def lanczos4(x):
    """Eq. (4): L(x; a) = sinc(x) sinc(x/a) on (-a, a), 0 elsewhere, with a = 4 and
    sinc(x) = sin(pi x) / (pi x) (np.sinc is exactly this normalised sinc)."""
    x = np.asarray(x, np.float64)
    return np.where(np.abs(x) < LANCZOS_A, np.sinc(x) * np.sinc(x / LANCZOS_A), 0.0)


def blur_taps(sigma: float, u):
    """Taps of the sheared-line Gaussian along direction u.

    Major axis = the coordinate with the larger |u| component; successive taps
    step one pixel along it and m pixels along the other axis (v = (1, m) or
    (m, 1)), so the line follows u exactly.  The Gaussian of standard
    deviation sigma (pixels) has sigma/|v| in units of taps; taps run
    k = -K..K with K = ceil(4 sigma/|v|); weights are normalised to sum 1."""
    ux, uy = u
    if abs(ux) >= abs(uy):
        major, m = 0, uy / ux
    else:
        major, m = 1, ux / uy
    sig_step = sigma / math.sqrt(1.0 + m * m)
    K = int(math.ceil(4.0 * sig_step))
    k = np.arange(-K, K + 1)
    g = np.exp(-(k.astype(np.float64) ** 2) / (2.0 * sig_step * sig_step))
    g /= g.sum()
    return major, m, k, g


def directional_blur(img, sigma: float, u):
    """Gaussian blur of standard deviation sigma along direction u, fp64 output.

    Each output pixel is sum_k g_k * I(p + k v); off-grid samples (the minor
    coordinate p_minor + k m) are linearly interpolated between the two
    neighbouring rows (or columns); all coordinates are clamped to the image
    (replicated border)."""
    I = np.asarray(img, np.float64)
    H, W = I.shape
    if sigma <= 0.0:
        return I.copy()
    major, m, ks, g = blur_taps(sigma, u)
    yy, xx = np.mgrid[0:H, 0:W]
    out = np.zeros((H, W), np.float64)
    for k, w in zip(ks, g):
        if major == 0:
            xk = np.clip(xx + k, 0, W - 1)
            yf = yy + k * m
            y0 = np.floor(yf)
            f = yf - y0
            y0 = y0.astype(np.int64)
            a = I[np.clip(y0, 0, H - 1), xk]
            b = I[np.clip(y0 + 1, 0, H - 1), xk]
        else:
            yk = np.clip(yy + k, 0, H - 1)
            xf = xx + k * m
            x0 = np.floor(xf)
            f = xf - x0
            x0 = x0.astype(np.int64)
            a = I[yk, np.clip(x0, 0, W - 1)]
            b = I[yk, np.clip(x0 + 1, 0, W - 1)]
        out += w * ((1.0 - f) * a + f * b)
    return out


def view_coords(view: View):
    """Source coordinates p = G(q) of every view pixel centre q (fp64), shape (H', W')."""
    qy, qx = np.mgrid[0:view.height, 0:view.width].astype(np.float64)
    G = view.inv
    px = G[0, 0] * qx + G[0, 1] * qy + G[0, 2]
    py = G[1, 0] * qx + G[1, 1] * qy + G[1, 2]
    return px, py


def valid_mask(view: View, px, py):
    """A view pixel holds image content iff its source point lies in [-1/2, W-1/2] x [-1/2, H-1/2]."""
    return (px >= -0.5) & (px <= view.src_w - 0.5) & (py >= -0.5) & (py <= view.src_h - 0.5)


def lanczos_sample(S, px, py):
    """Eq. (3) at the points (px, py): sum_j sum_i f(floor(x)+i, floor(y)+j) L(i - frac x) L(j - frac y),
    i, j = -3..4 (the 8x8 window of Sec. IV.C), divided by the sum of the weights so
    that constants are reproduced; taps outside the image are clamped to the border."""
    S = np.asarray(S, np.float64)
    H, W = S.shape
    ix = np.floor(px)
    iy = np.floor(py)
    fx = px - ix
    fy = py - iy
    ix = ix.astype(np.int64)
    iy = iy.astype(np.int64)
    taps = np.arange(-LANCZOS_A + 1, LANCZOS_A + 1)                  # -3..4
    wx = lanczos4(taps[None, :] - fx[:, None])                       # (n, 8)
    wy = lanczos4(taps[None, :] - fy[:, None])
    cols = np.clip(ix[:, None] + taps[None, :], 0, W - 1)            # (n, 8)
    rows = np.clip(iy[:, None] + taps[None, :], 0, H - 1)
    patch = S[rows[:, :, None], cols[:, None, :]]                    # (n, 8 rows, 8 cols)
    num = np.einsum("nj,ni,nji->n", wy, wx, patch)
    return num / (wx.sum(axis=1) * wy.sum(axis=1))


def warp_lanczos4(S, view: View, chunk: int = 1 << 16):
    """Resample source S (already anti-aliased) onto the view canvas.

    Returns (V, mask): V fp64 with 0 where the view pixel has no source
    content, mask bool."""
    px, py = view_coords(view)
    mask = valid_mask(view, px, py)
    V = np.zeros((view.height, view.width), np.float64)
    idx = np.flatnonzero(mask.ravel())
    fpx, fpy = px.ravel(), py.ravel()
    Vf = V.ravel()
    for a in range(0, idx.size, chunk):
        sl = idx[a:a + chunk]
        Vf[sl] = lanczos_sample(S, fpx[sl], fpy[sl])
    return V, mask


def nearest_sample(S, px, py):
    """Nearest-neighbour resampling (the paper's search-time interpolation, Sec. III): the
    source pixel floor(p + 1/2) on each axis (halves go up), clamped to the image."""
    S = np.asarray(S, np.float64)
    H, W = S.shape
    ix = np.clip(np.floor(px + 0.5).astype(np.int64), 0, W - 1)
    iy = np.clip(np.floor(py + 0.5).astype(np.int64), 0, H - 1)
    return S[iy, ix]


def warp_nearest(S, view: View):
    """Like warp_lanczos4 with nearest-neighbour sampling."""
    px, py = view_coords(view)
    mask = valid_mask(view, px, py)
    V = np.zeros((view.height, view.width), np.float64)
    V[mask] = nearest_sample(S, px[mask], py[mask])
    return V, mask


def quantize(V):
    """u8 = clamp(round-half-to-even(V), 0, 255)."""
    return np.clip(np.rint(V), 0, 255).astype(np.uint8)


def simulate_view(src_u8, view: View, interp: str = "lanczos4"):
    """One simulated view: blur along the tilt direction (t > 1), then Lanczos-4 resampling
    (interp = "lanczos4") or nearest-neighbour sampling (interp = "nearest").

    Returns (V fp64, mask bool, u8)."""
    S = directional_blur(src_u8, view.sigma, view.u) if view.sigma > 0 else np.asarray(src_u8, np.float64)
    V, mask = warp_nearest(S, view) if interp == "nearest" else warp_lanczos4(S, view)
    U = quantize(V)
    U[~mask] = 0
    return V, mask, U


def scale_image(src_u8, s: float):
    """Scale stage for the scale parameter of the sampling group (Sec. III.B): an isotropic
    anti-alias Gaussian of standard deviation 0.8 sqrt(1/s^2 - 1) for a reduction (s < 1;
    none for s >= 1), then Lanczos-4 resampling at p = (q + 1/2) / s - 1/2 onto a
    round(s W) x round(s H) grid, taps clamped to the image, rounded half to even.

    Returns (V fp64, u8).  The output grid is chosen so that every output pixel maps inside
    the source, and views of the scaled image use it as their source (s = 1 in their map)."""
    from .plan import scaled_size
    I = np.asarray(src_u8, np.float64)
    H, W = I.shape
    if s == 1.0:
        return I.copy(), np.asarray(src_u8, np.uint8).copy()
    if s < 1.0:
        sigma = 0.8 * math.sqrt(1.0 / (s * s) - 1.0)
        B = directional_blur(directional_blur(I, sigma, (1.0, 0.0)), sigma, (0.0, 1.0))
    else:
        B = I
    ws, hs = scaled_size(W, H, s)
    qy, qx = np.mgrid[0:hs, 0:ws].astype(np.float64)
    px = (qx + 0.5) / s - 0.5
    py = (qy + 0.5) / s - 0.5
    V = lanczos_sample(B, px.ravel(), py.ravel()).reshape(hs, ws)
    return V, quantize(V)
