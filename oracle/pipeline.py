"""The parameter-search hot path composed end to end on the CPU.

Test infrastructure only (see the package docstring).

Sec. III.B: simulate views of the images over the (t, phi) grid, run ORB on
every view, match views with a brute-force Hamming matcher and keep the view
pair with the most matches; the matched points of that pair are mapped back
to the original images (Sec. IV.B evaluates them with eqs. (5)-(6)).

Parity status: pinned.  The composed stages are pinned in their own modules; the back-map is
pinned by closed forms (the identity view maps level-0 keypoints to themselves, a level's pixel
centres span the view symmetrically, the scale-stage factor maps u to 2u + 1/2 at s = 1/2) and
by the view map (a back-mapped point maps forward onto its keypoint); end to end, the tiny pair's
matches agree with the known homography.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import match as M
from . import orb as O
from . import plan as P
from . import simulate as S


@dataclass
class OrbOptions:
    n_levels: int = 8
    scale: float = 1.2
    n_features: int = 1000
    fast_threshold: int = 20
    ratio_num: int = 4
    ratio_den: int = 5


def plan_image(w: int, h: int, grid, psi: float = 0.0, s: float = 1.0):
    """Views for grid entries (t, phi) or (t, phi, s) (the latter override s)."""
    return [P.plan_view(w, h, g[0], g[1], psi, g[2] if len(g) > 2 else s) for g in grid]


def simulate_image(src_u8, views, interp: str = "lanczos4"):
    """Per view (V fp64, mask, u8)."""
    return [S.simulate_view(src_u8, v, interp) for v in views]


def extract_image(sims, views, opts: OrbOptions, pattern):
    quotas = P.level_quotas(opts.n_features, opts.n_levels, opts.scale)
    feats = []
    for (V, mask, U), v in zip(sims, views):
        dims = P.level_dims(v.width, v.height, opts.n_levels, opts.scale)
        feats.append(O.extract_view(U, mask, dims, quotas, opts.fast_threshold, pattern))
    return feats


def keypoints_to_source(feat, view, opts: OrbOptions, src_scale: float = 1.0):
    """Keypoints -> coordinates of the original image (through the scale-stage factor)."""
    dims = P.level_dims(view.width, view.height, opts.n_levels, opts.scale)
    lw = np.array([d[0] for d in dims])
    lh = np.array([d[1] for d in dims])
    lv = feat["level"]
    x0, y0 = M.level_to_view(feat["x"], feat["y"], lw[lv], lh[lv], view.width, view.height)
    xs, ys = M.view_to_source(view, x0, y0)
    if src_scale != 1.0:
        xs, ys = (xs + 0.5) / src_scale - 0.5, (ys + 0.5) / src_scale - 0.5
    return xs, ys


def simulate_and_extract(img, grid, opts: OrbOptions, pattern, scales=(1.0,), interp: str = "lanczos4"):
    """Views of an image over the grid at every scale of the sampling group (Sec. III.B):
    scale s != 1 goes through the scale stage first and its views use s = 1 in their map
    (grid entries (t, phi, s) carry their own s into the view map instead)."""
    views, sims, feats, vscale = [], [], [], []
    for s in scales:
        src = img if s == 1.0 else S.scale_image(img, s)[1]
        vs = plan_image(src.shape[1], src.shape[0], grid)
        sm = simulate_image(src, vs, interp)
        views += vs
        sims += sm
        feats += extract_image(sm, vs, opts, pattern)
        vscale += [s] * len(vs)
    return views, sims, feats, vscale


def match_pair(A, B, grid_a, grid_b, opts: OrbOptions, pattern, scales_a=(1.0,), scales_b=(1.0,),
               interp: str = "lanczos4"):
    """Full path for one image pair.  Returns a dict with per-view features, the
    pair counts, the best pair and its accepted matches in original-image coordinates."""
    va, sa, fa, ka = simulate_and_extract(A, grid_a, opts, pattern, scales_a, interp)
    vb, sb, fb, kb = simulate_and_extract(B, grid_b, opts, pattern, scales_b, interp)
    results, counts, best = M.match_views([f["desc"] for f in fa], [f["desc"] for f in fb],
                                          opts.ratio_num, opts.ratio_den)
    k, i, j, c = best
    out = dict(views_a=va, views_b=vb, sims_a=sa, sims_b=sb, feats_a=fa, feats_b=fb,
               results=results, counts=counts, best=best)
    if k >= 0:
        idx, d1, d2, acc = results[k]
        qa = np.flatnonzero(acc)
        tb = idx[qa]
        xa, ya = keypoints_to_source(fa[i], va[i], opts, ka[i])
        xb, yb = keypoints_to_source(fb[j], vb[j], opts, kb[j])
        out["pa"] = np.stack([xa[qa], ya[qa]], axis=1)
        out["pb"] = np.stack([xb[tb], yb[tb]], axis=1)
    else:
        out["pa"] = np.zeros((0, 2))
        out["pb"] = np.zeros((0, 2))
    return out
