"""View planning: the sampling rule, the camera map and the view canvases.

Test infrastructure only (see the package docstring).

Parity status: pinned (view counts per tilt against the coefficients of
eq. (11); the printed best longitude of Sec. IV.D lies on the grid; identity
and quarter-turn canvases; anti-alias direction against the map).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Sec. III.B: tilts t = a^i with a = sqrt(2); longitudes k*b/t with b = 72 deg,
# k the largest natural number with k*b/t < 180 deg.
TILT_BASE = math.sqrt(2.0)
LONGITUDE_STEP_DEG = 72.0
# Anti-alias constant of the ASIFT construction the paper inherits its affine model from.
AA_C = 0.8


def tilt(i: int) -> float:
    """t_i = sqrt(2)^i, exact for even i (2^(i/2)), so that the k*b/t < 180 test
    is decided in exact arithmetic wherever it sits on the boundary."""
    return float(2 ** (i // 2)) * (math.sqrt(2.0) if i % 2 else 1.0)


def sampling_grid(n_tilt: int, b_deg: float = LONGITUDE_STEP_DEG):
    """List of (t, phi_radians) for tilt exponents 0..n_tilt (Sec. III.B sampling rule)."""
    out = []
    for i in range(n_tilt + 1):
        t = tilt(i)
        k = 0
        # k*b/t < 180  <=>  k*b < 180*t  (both sides exact for even i)
        while k * b_deg < 180.0 * t:
            out.append((t, math.radians(k * b_deg / t)))
            k += 1
    return out


def sampling_grid_scaled(n_tilt: int, delta_s: float, b_deg: float = LONGITUDE_STEP_DEG):
    """The search schedule of Sec. III.B with the scale tied to the tilt index:
    (t_i, phi, s_i) with s_i = 1 + i * delta_s (a magnification; eq. (11) charges the views
    of tilt index i the area factor (1 + i delta_s)^2)."""
    out = []
    for i in range(n_tilt + 1):
        t = tilt(i)
        for (tt, phi) in sampling_grid(i, b_deg):
            if tt == t:
                out.append((t, phi, 1.0 + i * delta_s))
    return out


def rot(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s], [s, c]], np.float64)


def linear_map(t: float, phi: float, psi: float = 0.0, s: float = 1.0) -> np.ndarray:
    """Source -> view linear map L = s R(psi) diag(1/t, 1) R(phi).

    Eq. (2) factors a camera change as T R1(psi) S T_tau R2(phi) with
    T_tau = diag(t, 1); read as the resampling map of ASIFT (the view is the
    source compressed by t along the axis that R2(phi) brings onto x), the
    source -> view direction carries diag(1/t, 1).  Scale s magnifies for s > 1."""
    return s * (rot(psi) @ np.diag([1.0 / t, 1.0]) @ rot(phi))


@dataclass
class View:
    t: float
    phi: float
    psi: float
    s: float
    src_w: int
    src_h: int
    width: int
    height: int
    fwd: np.ndarray      # 2x3: q = fwd[:, :2] @ p + fwd[:, 2]
    inv: np.ndarray      # 2x3: p = inv[:, :2] @ q + inv[:, 2]
    sigma: float         # anti-alias sigma (source pixels) along u, 0.8 sqrt((t/s)^2 - 1); 0 = none
    u: tuple             # unit direction in source coordinates compressed by the tilt


def plan_view(src_w: int, src_h: int, t: float, phi: float, psi: float = 0.0, s: float = 1.0,
              tx: float = 0.0, ty: float = 0.0) -> View:
    """Canvas and maps of one simulated view.

    The canvas is the bounding box of the source rectangle [-1/2, W-1/2] x
    [-1/2, H-1/2] under L, placed so that the box starts at -1/2 on the view
    grid; (tx, ty) of eq. (2) then shifts the content inside that canvas."""
    L = linear_map(t, phi, psi, s)
    corners = np.array([[-0.5, src_w - 0.5, -0.5, src_w - 0.5],
                        [-0.5, -0.5, src_h - 0.5, src_h - 0.5]], np.float64)
    mc = L @ corners
    lo = mc.min(axis=1)
    hi = mc.max(axis=1)
    width = int(math.ceil((hi[0] - lo[0]) - 1e-9))
    height = int(math.ceil((hi[1] - lo[1]) - 1e-9))
    tau = -lo - 0.5 + np.array([tx, ty])
    Li = np.linalg.inv(L)
    fwd = np.concatenate([L, tau[:, None]], axis=1)
    inv = np.concatenate([Li, (-Li @ tau)[:, None]], axis=1)
    # anti-alias for the net compression t/s along u (for s = 1 this is 0.8 sqrt(t^2 - 1))
    r = t / s
    sigma = AA_C * math.sqrt(r * r - 1.0) if r > 1.0 else 0.0
    # R(phi) maps this source direction onto the view's x axis, which diag(1/t, 1) compresses.
    u = (math.cos(phi), -math.sin(phi))
    return View(t, phi, psi, s, src_w, src_h, width, height, fwd, inv, sigma, u)


def level_dims(width: int, height: int, n_levels: int, scale: float = 1.2):
    """Pyramid level sizes: round(W / scale^l) (round half up), at least 1."""
    out = []
    for l in range(n_levels):
        f = scale ** l
        out.append((max(1, int(math.floor(width / f + 0.5))), max(1, int(math.floor(height / f + 0.5)))))
    return out


def level_quotas(n_features: int, n_levels: int, scale: float = 1.2):
    """Keypoints per level, proportional to level area: n_l = floor(N r_l / sum r),
    r_l = scale^(-2l), for l >= 1; level 0 takes the remainder."""
    r = [scale ** (-2 * l) for l in range(n_levels)]
    tot = 0.0
    for v in r:
        tot += v
    q = [0] * n_levels
    for l in range(1, n_levels):
        q[l] = int(math.floor(n_features * r[l] / tot))
    q[0] = n_features - sum(q[1:])
    return q


def scaled_size(width: int, height: int, s: float):
    """Size of the scale-stage image: round(s W), round(s H) (half up), at least 1."""
    return max(1, int(math.floor(s * width + 0.5))), max(1, int(math.floor(s * height + 0.5)))
