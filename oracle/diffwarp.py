"""The Lanczos-4 affine warp as a differentiable map of an fp image and of the six
camera parameters, and its adjoint.

Test infrastructure only (see the package docstring).

The warp is the resampling of eqs. (3)-(4) (8x8 window, weights normalised to
sum one, border taps clamped) driven by the camera map of eq. (2) with the
linear part L = s R(psi) diag(1/t, 1) R(phi) used everywhere in this package.
For photometric refinement of (t, phi) the crop keeps its size and the map
is centred: a view pixel q samples the image at

    p = L^-1 (q - c - T) + c,   c = ((w - 1)/2, (h - 1)/2),  T = (tx, ty),

so t = 1, phi = psi = 0, s = 1, T = 0 is the identity.  A view pixel is valid
iff p lies in [-1/2, w - 1/2] x [-1/2, h - 1/2]; invalid pixels are 0 and
carry no gradient.

The adjoint follows from the chain rule on the definition: with
Sx = sum_i wx_i, Sy = sum_j wy_j and V = sum_ij wx_i wy_j I_ij / (Sx Sy),

    dV/dI_ij  = wx_i wy_j / (Sx Sy)                       (summed over clamped copies)
    dV/dpx    = sum_ij wx'_i wy_j I_ij / (Sx Sy) - V Sx' / Sx,   wx'_i = -L'(i - fx)
    dV/dtheta = dV/dpx dpx/dtheta + dV/dpy dpy/dtheta

and dp/dtheta from differentiating L^-1 = (1/s) R(-phi) diag(t, 1) R(-psi).

Parity status: pinned.  The identity reproduces the image, integer shifts
reproduce shifted images, the kernel derivative equals a central difference
of np.sinc, the image adjoint passes the dot-product test <A x, y> = <x, A^T y>,
and the parameter gradient equals central finite differences of the forward
map in fp64.
"""
from __future__ import annotations

import math

import numpy as np

from .simulate import LANCZOS_A, lanczos4

PARAM_NAMES = ("t", "phi", "psi", "s", "tx", "ty")


def lanczos4_deriv(x):
    """d/dx of sinc(x) sinc(x/4) on (-4, 4), 0 elsewhere.

    With u = pi x: L = 4 sin(u) sin(u/4) / u^2, so
    L' = pi * 4 [cos(u) sin(u/4) + sin(u) cos(u/4) / 4 - 2 sin(u) sin(u/4) / u] / u^2.
    Near 0 the quotient cancels; there L' = -(17/48) pi^2 x + O(x^3)
    (from sinc(y) = 1 - (pi y)^2 / 6 + ...)."""
    x = np.asarray(x, np.float64)
    u = math.pi * x
    small = np.abs(x) < 1e-4
    us = np.where(small, 1.0, u)
    d = math.pi * 4.0 * (np.cos(us) * np.sin(us / 4) + np.sin(us) * np.cos(us / 4) / 4
                         - 2.0 * np.sin(us) * np.sin(us / 4) / us) / (us * us)
    d = np.where(small, -(17.0 / 48.0) * math.pi ** 2 * x, d)
    return np.where(np.abs(x) < LANCZOS_A, d, 0.0)


def rot(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s], [s, c]], np.float64)


J = np.array([[0.0, -1.0], [1.0, 0.0]])          # d/da R(a) = R(a) J


def inverse_linear(t, phi, psi, s):
    """M = L^-1 = (1/s) R(-phi) diag(t, 1) R(-psi)."""
    return (1.0 / s) * rot(-phi) @ np.diag([t, 1.0]) @ rot(-psi)


def inverse_linear_derivs(t, phi, psi, s):
    """dM/dt, dM/dphi, dM/dpsi, dM/ds."""
    M = inverse_linear(t, phi, psi, s)
    dt = (1.0 / s) * rot(-phi) @ np.diag([1.0, 0.0]) @ rot(-psi)
    dphi = (1.0 / s) * (-rot(-phi) @ J) @ np.diag([t, 1.0]) @ rot(-psi)
    dpsi = (1.0 / s) * rot(-phi) @ np.diag([t, 1.0]) @ (-rot(-psi) @ J)
    ds = -M / s
    return dt, dphi, dpsi, ds


def sample_points(params, w: int, h: int):
    """Source points p (px, py) of every view pixel, shape (h, w) each, and the valid mask."""
    t, phi, psi, s, tx, ty = (float(v) for v in params)
    M = inverse_linear(t, phi, psi, s)
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    qy, qx = np.mgrid[0:h, 0:w].astype(np.float64)
    dx, dy = qx - cx - tx, qy - cy - ty
    px = M[0, 0] * dx + M[0, 1] * dy + cx
    py = M[1, 0] * dx + M[1, 1] * dy + cy
    mask = (px >= -0.5) & (px <= w - 0.5) & (py >= -0.5) & (py <= h - 0.5)
    return px, py, dx, dy, mask


def _taps(img, px, py):
    H, W = img.shape
    ix, iy = np.floor(px), np.floor(py)
    fx, fy = px - ix, py - iy
    k = np.arange(-LANCZOS_A + 1, LANCZOS_A + 1)                      # -3..4
    wx = lanczos4(k[None, :] - fx[:, None])
    wy = lanczos4(k[None, :] - fy[:, None])
    dwx = -lanczos4_deriv(k[None, :] - fx[:, None])                  # d wx / d px
    dwy = -lanczos4_deriv(k[None, :] - fy[:, None])
    cols = np.clip(ix.astype(np.int64)[:, None] + k[None, :], 0, W - 1)
    rows = np.clip(iy.astype(np.int64)[:, None] + k[None, :], 0, H - 1)
    return wx, wy, dwx, dwy, rows, cols


def warp_forward(img, params):
    """V (fp64, h x w) and the valid mask for one crop."""
    I = np.asarray(img, np.float64)
    h, w = I.shape
    px, py, _, _, mask = sample_points(params, w, h)
    V = np.zeros((h, w))
    sel = mask.ravel()
    wx, wy, _, _, rows, cols = _taps(I, px.ravel()[sel], py.ravel()[sel])
    patch = I[rows[:, :, None], cols[:, None, :]]
    V.ravel()[sel] = np.einsum("nj,ni,nji->n", wy, wx, patch) / (wx.sum(1) * wy.sum(1))
    return V, mask


def warp_adjoint(img, gout, params):
    """(dLoss/dimg, dLoss/dparams[6]) for dLoss/dV = gout."""
    I = np.asarray(img, np.float64)
    G = np.asarray(gout, np.float64)
    h, w = I.shape
    px, py, dx, dy, mask = sample_points(params, w, h)
    sel = mask.ravel()
    g = G.ravel()[sel]
    wx, wy, dwx, dwy, rows, cols = _taps(I, px.ravel()[sel], py.ravel()[sel])
    Sx, Sy = wx.sum(1), wy.sum(1)
    norm = 1.0 / (Sx * Sy)
    # image: scatter g * wx_i wy_j / (Sx Sy) to the (clamped) taps
    contrib = g[:, None, None] * wy[:, :, None] * wx[:, None, :] * norm[:, None, None]
    gimg = np.zeros(h * w)
    np.add.at(gimg, (rows[:, :, None] * w + cols[:, None, :]).ravel(), contrib.ravel())
    # geometry
    patch = I[rows[:, :, None], cols[:, None, :]]
    V = np.einsum("nj,ni,nji->n", wy, wx, patch) * norm
    dV_dpx = np.einsum("nj,ni,nji->n", wy, dwx, patch) * norm - V * dwx.sum(1) / Sx
    dV_dpy = np.einsum("nj,ni,nji->n", dwy, wx, patch) * norm - V * dwy.sum(1) / Sy
    t, phi, psi, s, tx, ty = (float(v) for v in params)
    M = inverse_linear(t, phi, psi, s)
    ddx, ddy = dx.ravel()[sel], dy.ravel()[sel]
    gp = np.zeros(6)
    for k, D in enumerate(inverse_linear_derivs(t, phi, psi, s)):
        dpx = D[0, 0] * ddx + D[0, 1] * ddy
        dpy = D[1, 0] * ddx + D[1, 1] * ddy
        gp[k] = np.sum(g * (dV_dpx * dpx + dV_dpy * dpy))
    # d(q - c - T)/dtx = (-1, 0), /dty = (0, -1)
    gp[4] = np.sum(g * (dV_dpx * -M[0, 0] + dV_dpy * -M[1, 0]))
    gp[5] = np.sum(g * (dV_dpx * -M[0, 1] + dV_dpy * -M[1, 1]))
    return gimg.reshape(h, w), gp


def l2_loss_and_grads(img, target, params):
    """Photometric loss 1/2 sum over valid pixels (V - target)^2 and its gradients."""
    V, mask = warp_forward(img, params)
    r = np.where(mask, V - np.asarray(target, np.float64), 0.0)
    gimg, gp = warp_adjoint(img, r, params)
    return 0.5 * float(np.sum(r * r)), gimg, gp
