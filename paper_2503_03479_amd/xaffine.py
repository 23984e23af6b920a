"""ctypes binding of libxaffine (include/xaffine.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  If the
library is missing the import of this module still works, but every call
raises RuntimeError (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxaffine.so")

XA_OK, XA_EINVAL, XA_ECAPACITY, XA_EHIP, XA_EUNSUPPORTED = 0, -1, -2, -3, -4
STATUS_NAMES = {0: "XA_OK", -1: "XA_EINVAL", -2: "XA_ECAPACITY", -3: "XA_EHIP", -4: "XA_EUNSUPPORTED"}
DESC_BYTES = 32

# numpy mirrors of the C structs
PARAMS_DTYPE = np.dtype([("t", "f8"), ("phi", "f8"), ("psi", "f8"), ("s", "f8"), ("tx", "f8"), ("ty", "f8")])
SOURCE_DTYPE = np.dtype([("width", "i4"), ("height", "i4"), ("pitch", "i4"), ("pad", "i4"), ("offset", "i8"),
                         ("scale", "f8")])
VIEW_DTYPE = np.dtype([("p", PARAMS_DTYPE), ("source", "i4"), ("src_w", "i4"), ("src_h", "i4"), ("src_pitch", "i4"),
                       ("src_offset", "i8"), ("src_scale", "f8"), ("width", "i4"), ("height", "i4"), ("pitch", "i4"),
                       ("warp_tile_w", "i4"), ("fwd", "f8", 6), ("inv", "f8", 6), ("sigma", "f8"), ("ux", "f8"),
                       ("uy", "f8"), ("offset", "i8"), ("blur_offset", "i8"), ("blur_major", "i4"), ("blur_tap0", "i4"),
                       ("blur_ntaps", "i4"), ("interp", "i4"), ("warp_ls_mod", "i4"), ("blur_rows", "i4")])
LEVEL_DTYPE = np.dtype([("width", "i4"), ("height", "i4"), ("pitch", "i4"), ("quota", "i4"), ("offset", "i8"),
                        ("kp_base", "i4"), ("view", "i4"), ("level", "i4"), ("pad", "i4"), ("cand_offset", "i8"),
                        ("cand_cap", "i8")])
HEADER_DTYPE = np.dtype([("magic", "u4"), ("version", "u4"), ("src_w", "i4"), ("src_h", "i4"), ("n_views", "i4"),
                         ("n_levels", "i4"), ("n_features", "i4"), ("fast_threshold", "i4"), ("level_scale", "f8"),
                         ("total_bytes", "i8"), ("arena_bytes", "i8"), ("cand_total", "i8"), ("blur_floats", "i8"),
                         ("n_blur", "i4"), ("n_taps_total", "i4"), ("off_views", "i8"), ("off_levels", "i8"),
                         ("off_taps", "i8"), ("off_blur_views", "i8"), ("off_warp_prefix", "i8"),
                         ("off_level_prefix", "i8"), ("off_vl_prefix", "i8"), ("off_blur_prefix", "i8"),
                         ("off_sources", "i8"), ("n_sources", "i4"), ("pad", "i4"), ("off_fast_flags", "i8")])
TAP_DTYPE = np.dtype([("wa", "f4"), ("wb", "f4"), ("dmaj", "i4"), ("dmin", "i4")])
KEYPOINT_DTYPE = np.dtype([("x", "i4"), ("y", "i4"), ("level", "i4"), ("bin", "i4"), ("harris", "i8"),
                           ("xs", "f8"), ("ys", "f8")])
MATCH_DTYPE = np.dtype([("t", "i4"), ("d1", "u2"), ("d2", "u2")])
assert VIEW_DTYPE.itemsize == 256 and LEVEL_DTYPE.itemsize == 56 and KEYPOINT_DTYPE.itemsize == 40
assert MATCH_DTYPE.itemsize == 8 and HEADER_DTYPE.itemsize == 168 and SOURCE_DTYPE.itemsize == 32


class XAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("t", "phi", "psi", "s", "tx", "ty")]


class _BatchBuffers(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("kp", "desc", "count", "matches", "pair_count", "best")]


class _PairBuffers(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("kp_a", "desc_a", "count_a", "kp_b", "desc_b", "count_b",
                                                 "matches", "pair_count", "best")]


_c = ctypes
_SIGS = {
    "xa_last_error": (_c.c_char_p, []),
    "xa_version": (_c.c_char_p, []),
    "xa_sampling_grid": (_c.c_int, [_c.c_int32, _c.c_double, _c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32)]),
    "xa_plan_views": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32,
                                 _c.c_double, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_size_t,
                                 _c.POINTER(_c.c_size_t)]),
    "xa_plan_image": (_c.c_int, [_c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_int32, _c.c_int32, _c.c_double,
                                 _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_size_t, _c.POINTER(_c.c_size_t)]),
    "xa_scaled_size": (_c.c_int, [_c.c_int32, _c.c_int32, _c.c_double, _c.POINTER(_c.c_int32),
                                  _c.POINTER(_c.c_int32)]),
    "xa_plan_scales": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_size_t, _c.POINTER(_c.c_size_t)]),
    "xa_scale_workspace_size": (_c.c_size_t, [_c.c_void_p]),
    "xa_scale_sources": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                    _c.c_void_p]),
    "xa_simulate_workspace_size": (_c.c_size_t, [_c.c_void_p]),
    "xa_simulate_views": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                     _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_blur_views": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_warp_views": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                 _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_extract_workspace_size": (_c.c_size_t, [_c.c_void_p]),
    "xa_extract_orb": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_match_views": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_int32,
                                  _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p]),
    "xa_plan_matches": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_size_t,
                                   _c.POINTER(_c.c_size_t)]),
    "xa_match_groups": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32,
                                   _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "xa_match_l2_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32]),
    "xa_match_l2": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p,
                               _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_match_l2_noalloc": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32,
                                       _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "xa_sift_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32, _c.c_void_p]),
    "xa_extract_sift": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                   _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_sift_match_points": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32,
                                        _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                        _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "xa_scaling_coefficient_f64": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32,
                                              _c.c_void_p, _c.c_void_p]),
    "xa_set_warp_tiles": (_c.c_int, [_c.c_void_p]),
    "xa_get_warp_tiles": (_c.c_int, [_c.c_void_p]),
    "xa_tune_warp_tiles_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32]),
    "xa_tune_warp_tiles": (_c.c_int, [_c.c_int32, _c.c_int32, _c.c_void_p, _c.c_size_t, _c.c_void_p, _c.c_void_p,
                                      _c.c_void_p]),
    "xa_set_blur_rows": (_c.c_int, [_c.c_void_p]),
    "xa_get_blur_rows": (_c.c_int, [_c.c_void_p]),
    "xa_tune_blur_rows_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32]),
    "xa_tune_blur_rows": (_c.c_int, [_c.c_int32, _c.c_int32, _c.c_void_p, _c.c_size_t, _c.c_void_p, _c.c_void_p,
                                     _c.c_void_p]),
    "xa_tune_matcher_workspace_size": (_c.c_size_t, [_c.c_void_p, _c.c_int32, _c.c_int32]),
    "xa_tune_matcher": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_int32,
                                   _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                   _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "xa_blur_f32_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32, _c.c_int32]),
    "xa_blur_f32": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_double, _c.c_void_p,
                               _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_match_batch_workspace_size": (_c.c_size_t, [_c.c_void_p, _c.c_int32, _c.c_void_p]),
    "xa_match_batch": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32, _c.c_void_p,
                                  _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_match_batch_capture": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                          _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32,
                                          _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                          _c.POINTER(_c.c_void_p)]),
    "xa_graph_launch": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "xa_graph_destroy": (_c.c_int, [_c.c_void_p]),
    "xa_warp_f32_fwd_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32, _c.c_int32]),
    "xa_warp_f32_fwd": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                   _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_warp_f32_bwd_workspace_size": (_c.c_size_t, [_c.c_int32, _c.c_int32, _c.c_int32]),
    "xa_warp_f32_bwd": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32, _c.c_int32,
                                   _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_sampling_grid_scaled": (_c.c_int, [_c.c_int32, _c.c_double, _c.c_double, _c.c_void_p, _c.c_int32,
                                           _c.POINTER(_c.c_int32)]),
    "xa_plan_set_interp": (_c.c_int, [_c.c_void_p, _c.c_int32]),
    "xa_best_pair_points": (_c.c_int, [_c.c_void_p] * 5 + [_c.c_int32] * 4 + [_c.c_void_p] * 6),
    "xa_scaling_coefficient": (_c.c_int, [_c.c_void_p] * 4 + [_c.c_int32, _c.c_void_p, _c.c_void_p]),
    "xa_ransac_homography": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_int32, _c.c_double,
                                        _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "xa_match_pair_workspace_size": (_c.c_size_t, [_c.c_void_p, _c.c_void_p]),
    "xa_match_pair": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                 _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32,
                                 _c.POINTER(_PairBuffers), _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "xa_check": (_c.c_int, [_c.c_void_p]),
    "xa_pair_precision": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32,
                                     _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_double,
                                     _c.c_void_p, _c.c_void_p]),
}
EXPORTS = tuple(_SIGS)

_lib = None


def lib():
    """The loaded library; raises RuntimeError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2503_03479_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != XA_OK:
        raise XAError(status, lib().xa_last_error().decode())


def version() -> str:
    return lib().xa_version().decode()


# ---------------------------------------------------------------- planning (host only)

def sampling_grid(n_tilt: int, b_deg: float = 72.0, delta_s: float = 0.0) -> np.ndarray:
    """The (t, phi) grid of Sec. III.B; delta_s > 0 ties the scale to the tilt index, s = 1 + i delta_s."""
    n = ctypes.c_int32(0)
    st = lib().xa_sampling_grid_scaled(n_tilt, b_deg, delta_s, None, 0, ctypes.byref(n))
    if st not in (XA_OK, XA_ECAPACITY):
        _check(st)
    out = np.zeros(n.value, PARAMS_DTYPE)
    _check(lib().xa_sampling_grid_scaled(n_tilt, b_deg, delta_s, out.ctypes.data, n.value, ctypes.byref(n)))
    return out


INTERP = {"lanczos4": 0, "nearest": 1}


WARP_CLASSES = 8
WARP_CANDIDATES = (4, 8, 16, 32, 64)
_TUNED_TILES = {}        # device name -> widths chosen by tune_warp_tiles in this process


def set_warp_tiles(widths=None):
    """Warp tile widths per compression class for plans made from now on (None: the built-in rule)."""
    if widths is None:
        _check(lib().xa_set_warp_tiles(None))
        return
    w = np.ascontiguousarray(widths, np.int32)
    if w.shape != (WARP_CLASSES,):
        raise XAError(-1, f"need {WARP_CLASSES} widths")
    _check(lib().xa_set_warp_tiles(w.ctypes.data))


def get_warp_tiles() -> np.ndarray:
    w = np.zeros(WARP_CLASSES, np.int32)
    _check(lib().xa_get_warp_tiles(w.ctypes.data))
    return w


def tune_warp_tiles(device="cuda", src_w: int = 1024, src_h: int = 768, apply: bool = True, cache: bool = True):
    """Run the library's warp tile tuner (xa_tune_warp_tiles) on `device`; returns (widths int32
    [classes], ms float32 [classes, candidates]).  With apply, the widths are set for the plans
    made from then on; with cache, a device already tuned in this process is not timed again
    (ms is then None)."""
    import torch
    dev = torch.device(device)
    name = torch.cuda.get_device_name(dev)
    if cache and name in _TUNED_TILES:
        widths, ms = _TUNED_TILES[name], None
    else:
        need = lib().xa_tune_warp_tiles_workspace_size(src_w, src_h)
        if need == 0:
            raise XAError(-1, "tuning image size out of range")
        ws = _empty(need, dev)
        widths = np.zeros(WARP_CLASSES, np.int32)
        ms = np.zeros((WARP_CLASSES, len(WARP_CANDIDATES)), np.float32)
        with torch.cuda.device(dev):
            _check(lib().xa_tune_warp_tiles(src_w, src_h, _ptr(ws), ws.numel(), _stream(), widths.ctypes.data,
                                            ms.ctypes.data))
        _TUNED_TILES[name] = widths.copy()
    if apply:
        set_warp_tiles(widths)
    return widths, ms


BLUR_ROWS = (4, 8)
_TUNED_ROWS = {}         # device name -> blur rows chosen by tune_blur_rows in this process


def set_blur_rows(rows=None):
    """Blur outputs per thread (4 or 8) per compression class for plans made from now on (None: 8)."""
    if rows is None:
        _check(lib().xa_set_blur_rows(None))
        return
    r = np.ascontiguousarray(rows, np.int32)
    if r.shape != (WARP_CLASSES,):
        raise XAError(-1, f"need {WARP_CLASSES} values")
    _check(lib().xa_set_blur_rows(r.ctypes.data))


def get_blur_rows() -> np.ndarray:
    r = np.zeros(WARP_CLASSES, np.int32)
    _check(lib().xa_get_blur_rows(r.ctypes.data))
    return r


def tune_blur_rows(device="cuda", src_w: int = 1024, src_h: int = 768, apply: bool = True, cache: bool = True):
    """Run the library's blur tuner (xa_tune_blur_rows) on `device`; returns (rows int32 [classes],
    ms float32 [classes, 2] for 4 and 8 rows).  apply and cache as for tune_warp_tiles."""
    import torch
    dev = torch.device(device)
    name = torch.cuda.get_device_name(dev)
    if cache and name in _TUNED_ROWS:
        rows, ms = _TUNED_ROWS[name], None
    else:
        need = lib().xa_tune_blur_rows_workspace_size(src_w, src_h)
        if need == 0:
            raise XAError(-1, "tuning image size out of range")
        ws = _empty(need, dev)
        rows = np.zeros(WARP_CLASSES, np.int32)
        ms = np.zeros((WARP_CLASSES, len(BLUR_ROWS)), np.float32)
        with torch.cuda.device(dev):
            _check(lib().xa_tune_blur_rows(src_w, src_h, _ptr(ws), ws.numel(), _stream(), rows.ctypes.data,
                                           ms.ctypes.data))
        _TUNED_ROWS[name] = rows.copy()
    if apply:
        set_blur_rows(rows)
    return rows, ms


def _set_interp(plan: "Plan", interp: str) -> "Plan":
    if interp not in INTERP:
        raise XAError(-1, f"interp must be one of {sorted(INTERP)}")
    if INTERP[interp] != 0:
        _check(lib().xa_plan_set_interp(plan.blob.ctypes.data, INTERP[interp]))
    return _wrap_plan(plan.blob)


def make_params(rows) -> np.ndarray:
    """Params array from (t, phi[, psi, s, tx, ty]) tuples."""
    out = np.zeros(len(rows), PARAMS_DTYPE)
    for i, r in enumerate(rows):
        r = tuple(r) + (0.0, 1.0, 0.0, 0.0)[len(r) - 2:]
        out[i] = r[:6]
    return out


@dataclass
class Plan:
    blob: np.ndarray          # uint8 host bytes
    header: np.void
    views: np.ndarray         # VIEW_DTYPE
    levels: np.ndarray        # LEVEL_DTYPE, (n_views, n_levels)
    _dev: object = None

    @property
    def n_views(self) -> int:
        return int(self.header["n_views"])

    @property
    def n_levels(self) -> int:
        return int(self.header["n_levels"])

    @property
    def n_features(self) -> int:
        return int(self.header["n_features"])

    @property
    def arena_bytes(self) -> int:
        return int(self.header["arena_bytes"])

    def host_ptr(self) -> int:
        return self.blob.ctypes.data

    def device(self, device="cuda"):
        """Device copy of the blob (cached)."""
        import torch
        want = torch.device(device)
        if want.type == "cuda" and want.index is None:
            want = torch.device("cuda", torch.cuda.current_device())
        if self._dev is None or self._dev.device != want:
            self._dev = torch.from_numpy(self.blob.copy()).to(want)
        return self._dev

    def taps(self) -> np.ndarray:
        h = self.header
        return np.frombuffer(self.blob, TAP_DTYPE, int(h["n_taps_total"]), int(h["off_taps"]))

    def level_image(self, arena: np.ndarray, view: int, level: int) -> np.ndarray:
        """(H, W) view of one level inside a host copy of an arena (u8 or the fp32 values)."""
        L = self.levels[view, level]
        o, w, h, p = int(L["offset"]), int(L["width"]), int(L["height"]), int(L["pitch"])
        return arena[o:o + p * h].reshape(h, p)[:, :w]


def _wrap_plan(blob: np.ndarray) -> Plan:
    h = np.frombuffer(blob, HEADER_DTYPE, 1)[0]
    views = np.frombuffer(blob, VIEW_DTYPE, int(h["n_views"]), int(h["off_views"]))
    levels = np.frombuffer(blob, LEVEL_DTYPE, int(h["n_views"]) * int(h["n_levels"]),
                           int(h["off_levels"])).reshape(int(h["n_views"]), int(h["n_levels"]))
    return Plan(blob, h, views, levels)


def plan_views(sources: np.ndarray, view_source, params: np.ndarray, n_levels: int = 8, level_scale: float = 1.2,
               n_features: int = 1000, fast_threshold: int = 20, interp: str = "lanczos4") -> Plan:
    """Plan views of several sources (SOURCE_DTYPE array); view i simulates sources[view_source[i]]."""
    sources = np.ascontiguousarray(sources, SOURCE_DTYPE)
    vs = np.ascontiguousarray(view_source, np.int32)
    params = np.ascontiguousarray(params, PARAMS_DTYPE)
    assert len(vs) == len(params)
    n = ctypes.c_size_t(0)
    args = (sources.ctypes.data, len(sources), vs.ctypes.data, params.ctypes.data, len(params), n_levels, level_scale,
            n_features, fast_threshold)
    _check(lib().xa_plan_views(*args, None, 0, ctypes.byref(n)))
    blob = np.zeros(n.value, np.uint8)
    _check(lib().xa_plan_views(*args, blob.ctypes.data, blob.size, ctypes.byref(n)))
    return _set_interp(_wrap_plan(blob), interp)


def plan_image(src_w: int, src_h: int, params: np.ndarray, n_levels: int = 8, level_scale: float = 1.2,
               n_features: int = 1000, fast_threshold: int = 20, src_pitch: int | None = None,
               interp: str = "lanczos4") -> Plan:
    """Plan views of one image stored at offset 0 of its buffer with the given row pitch."""
    params = np.ascontiguousarray(params, PARAMS_DTYPE)
    pitch = src_w if src_pitch is None else src_pitch
    n = ctypes.c_size_t(0)
    args = (src_w, src_h, pitch, params.ctypes.data, len(params), n_levels, level_scale, n_features, fast_threshold)
    _check(lib().xa_plan_image(*args, None, 0, ctypes.byref(n)))
    blob = np.zeros(n.value, np.uint8)
    _check(lib().xa_plan_image(*args, blob.ctypes.data, blob.size, ctypes.byref(n)))
    return _set_interp(_wrap_plan(blob), interp)


SCALE_JOB_DTYPE = np.dtype([("src", SOURCE_DTYPE), ("dst", SOURCE_DTYPE), ("s", "f8")])


def scaled_size(w: int, h: int, s: float):
    ow, oh = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().xa_scaled_size(w, h, s, ctypes.byref(ow), ctypes.byref(oh)))
    return ow.value, oh.value


@dataclass
class ScalePlan:
    blob: np.ndarray
    jobs: np.ndarray
    _dev: object = None

    def host_ptr(self) -> int:
        return self.blob.ctypes.data

    def device(self, device="cuda"):
        import torch
        if self._dev is None:
            self._dev = torch.from_numpy(self.blob.copy()).to(device)
        return self._dev


def plan_scales(jobs: np.ndarray) -> ScalePlan:
    jobs = np.ascontiguousarray(jobs, SCALE_JOB_DTYPE)
    n = ctypes.c_size_t(0)
    _check(lib().xa_plan_scales(jobs.ctypes.data, len(jobs), None, 0, ctypes.byref(n)))
    blob = np.zeros(n.value, np.uint8)
    _check(lib().xa_plan_scales(jobs.ctypes.data, len(jobs), blob.ctypes.data, blob.size, ctypes.byref(n)))
    return ScalePlan(blob, jobs)


class SourceArena:
    """Host-side layout of a sources buffer: images appended at 256-byte aligned offsets with
    16-byte aligned pitches, plus scale-stage outputs."""

    def __init__(self):
        self.descs = []
        self.size = 0

    def add(self, width: int, height: int, scale: float = 1.0) -> int:
        pitch = (width + 15) // 16 * 16
        off = (self.size + 255) // 256 * 256
        self.descs.append((width, height, pitch, 0, off, scale))
        self.size = off + pitch * height
        return len(self.descs) - 1

    def table(self) -> np.ndarray:
        return np.array(self.descs, SOURCE_DTYPE)

    def pack(self, images: dict) -> np.ndarray:
        """Host buffer with the given {index: uint8 image} written at their offsets."""
        buf = np.zeros(max(self.size, 1), np.uint8)
        for i, img in images.items():
            w, h, p, _, o, _ = self.descs[i]
            buf[o:o + p * h].reshape(h, p)[:, :w] = img
        return buf

    def view(self, buf: np.ndarray, i: int) -> np.ndarray:
        w, h, p, _, o, _ = self.descs[i]
        return buf[o:o + p * h].reshape(h, p)[:, :w]


def scale_sources(splan: ScalePlan, sources, values: bool = False, ws=None):
    """Run the scale stage in place on a device sources buffer; optional fp32 values (same offsets)."""
    import torch
    dev = sources.device
    vals = torch.zeros(sources.numel(), dtype=torch.float32, device=dev) if values else None
    need = lib().xa_scale_workspace_size(splan.host_ptr())
    if ws is None:
        ws = _empty(need, dev)
    _check(lib().xa_scale_sources(splan.host_ptr(), _ptr(splan.device(dev)), _ptr(sources), _ptr(vals), _ptr(ws),
                                  ws.numel(), _stream()))
    return vals


# ---------------------------------------------------------------- device calls

def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def _empty(nbytes: int, device):
    import torch
    # 256-byte aligned (torch's caching allocator aligns to at least 512 bytes)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def simulate_views(plan: Plan, src, values: bool = False, ws=None):
    """Returns (arena u8, mask u8[, values f32]) device tensors of arena_bytes elements."""
    import torch
    dev = src.device
    assert src.dtype == torch.uint8 and src.is_contiguous()
    arena = torch.zeros(plan.arena_bytes, dtype=torch.uint8, device=dev)
    mask = torch.zeros(plan.arena_bytes, dtype=torch.uint8, device=dev)
    vals = torch.zeros(plan.arena_bytes, dtype=torch.float32, device=dev) if values else None
    need = lib().xa_simulate_workspace_size(plan.host_ptr())
    if ws is None:
        ws = _empty(need, dev)
    _check(lib().xa_simulate_views(plan.host_ptr(), _ptr(plan.device(dev)), _ptr(src), _ptr(arena),
                                   _ptr(mask), _ptr(vals), _ptr(ws), ws.numel(), _stream()))
    return (arena, mask, vals) if values else (arena, mask)


def blur_views(plan: Plan, src, ws):
    """First stage of simulate_views: the blurred fp32 planes of the plan's blurred views, into ws
    (xa_simulate_workspace_size bytes)."""
    _check(lib().xa_blur_views(plan.host_ptr(), _ptr(plan.device(src.device)), _ptr(src), _ptr(ws), ws.numel(),
                               _stream()))


def warp_views(plan: Plan, src, arena, mask, ws, values=None):
    """Second stage of simulate_views: every view resampled from the planes blur_views left in ws."""
    _check(lib().xa_warp_views(plan.host_ptr(), _ptr(plan.device(src.device)), _ptr(src), _ptr(arena), _ptr(mask),
                               _ptr(values), _ptr(ws), ws.numel(), _stream()))


def extract_orb(plan: Plan, arena, mask, pattern, ws=None):
    """ORB on every view.  Returns (kp u8[n_views, N, 40], desc u8[n_views, N, 32], count i32[n_views])."""
    import torch
    dev = arena.device
    N = plan.n_features
    kp = torch.zeros((plan.n_views, N, KEYPOINT_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    desc = torch.zeros((plan.n_views, N, DESC_BYTES), dtype=torch.uint8, device=dev)
    count = torch.zeros(plan.n_views, dtype=torch.int32, device=dev)
    need = lib().xa_extract_workspace_size(plan.host_ptr())
    if ws is None:
        ws = _empty(need, dev)
    _check(lib().xa_extract_orb(plan.host_ptr(), _ptr(plan.device(dev)), _ptr(arena), _ptr(mask), _ptr(pattern),
                                _ptr(kp), _ptr(desc), _ptr(count), _ptr(ws), ws.numel(), _stream()))
    return kp, desc, count


def match_views(desc_a, count_a, desc_b, count_b, ratio_num: int = 4, ratio_den: int = 5):
    """All-pairs matching.  Returns (matches u8[n_a*n_b, N, 8], pair_count i32[n_a*n_b], best i32[4])."""
    import torch
    dev = desc_a.device
    n_a, N = desc_a.shape[0], desc_a.shape[1]
    n_b = desc_b.shape[0]
    matches = torch.zeros((n_a * n_b, N, MATCH_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    pair_count = torch.zeros(n_a * n_b, dtype=torch.int32, device=dev)
    best = torch.zeros(4, dtype=torch.int32, device=dev)
    _check(lib().xa_match_views(_ptr(desc_a), _ptr(count_a), n_a, _ptr(desc_b), _ptr(count_b), n_b, N, ratio_num,
                                ratio_den, _ptr(matches), _ptr(pair_count), _ptr(best), _stream()))
    return matches, pair_count, best


class PairRunner:
    """Preallocated buffers for repeated xa_match_pair calls on images of fixed sizes."""

    def __init__(self, plan_a: Plan, plan_b: Plan, device="cuda"):
        import torch
        self.plan_a, self.plan_b = plan_a, plan_b
        self.device = torch.device(device)
        N = plan_a.n_features
        na, nb = plan_a.n_views, plan_b.n_views
        z = lambda *s, dt=torch.uint8: torch.zeros(s, dtype=dt, device=self.device)  # noqa: E731
        self.kp_a, self.desc_a, self.count_a = z(na, N, 40), z(na, N, 32), z(na, dt=torch.int32)
        self.kp_b, self.desc_b, self.count_b = z(nb, N, 40), z(nb, N, 32), z(nb, dt=torch.int32)
        self.matches, self.pair_count = z(na * nb, N, 8), z(na * nb, dt=torch.int32)
        self.best = z(4, dt=torch.int32)
        need = lib().xa_match_pair_workspace_size(plan_a.host_ptr(), plan_b.host_ptr())
        self.ws = _empty(need, self.device)
        self.bufs = _PairBuffers(*[_ptr(t) for t in (self.kp_a, self.desc_a, self.count_a, self.kp_b, self.desc_b,
                                                     self.count_b, self.matches, self.pair_count, self.best)])
        self.dev_a = plan_a.device(self.device)
        self.dev_b = plan_b.device(self.device)

    def run(self, A, B, pattern, ratio_num: int = 4, ratio_den: int = 5):
        _check(lib().xa_match_pair(self.plan_a.host_ptr(), _ptr(self.dev_a), _ptr(A),
                                   self.plan_b.host_ptr(), _ptr(self.dev_b), _ptr(B), _ptr(pattern),
                                   ratio_num, ratio_den, ctypes.byref(self.bufs), _ptr(self.ws), self.ws.numel(),
                                   _stream()))

    def precision(self, H, th: float = 2.0, ratio_num: int = 4, ratio_den: int = 5):
        import torch
        out = torch.zeros(2, dtype=torch.int32, device=self.device)
        Hc = np.ascontiguousarray(H, np.float64).reshape(9)
        _check(lib().xa_pair_precision(_ptr(self.kp_a), _ptr(self.kp_b), _ptr(self.matches), _ptr(self.count_a),
                                       _ptr(self.count_b), self.plan_b.n_views, self.plan_a.n_features, ratio_num,
                                       ratio_den, _ptr(self.best), Hc.ctypes.data, th, _ptr(out), _stream()))
        return out


def keypoints_np(kp_tensor) -> np.ndarray:
    """Device keypoint buffer -> numpy structured array (n_views, N)."""
    a = kp_tensor.cpu().numpy()
    return a.reshape(a.shape[0], a.shape[1] * a.shape[2]).view(KEYPOINT_DTYPE)


L2_MATCH_DTYPE = np.dtype([("t", "i4"), ("d1", "u4"), ("d2", "u4")])
L2_MISSING = 0xFFFFFFFF


def match_l2(dq, dt, ratio_num: int = 3, ratio_den: int = 4, ws=None):
    """Exact L2 nearest-two matching of 8-bit SIFT descriptors (xa_match_l2): dq [n_q, 128] and
    dt [n_t, 128] uint8 device tensors.  Returns (out int32 [n_q, 3] = (t, d1, d2) with d1, d2 the
    squared distances as uint32 bits, count int32 [1] of ratio-test passes); decode with
    l2_matches_np."""
    import torch
    for name, d in (("dq", dq), ("dt", dt)):
        if d.dtype != torch.uint8 or d.dim() != 2 or d.shape[1] != 128 or not d.is_contiguous():
            raise ValueError(f"{name} must be a contiguous uint8 tensor of shape [n, 128]")
    dev = dq.device
    nq, nt = int(dq.shape[0]), int(dt.shape[0])
    need = lib().xa_match_l2_workspace_size(nq, nt)
    if ws is None:
        ws = _empty(need, dev)
    out = torch.empty((max(nq, 1), 3), dtype=torch.int32, device=dev)
    count = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().xa_match_l2(_ptr(dq) if nq else None, nq, _ptr(dt) if nt else None, nt, ratio_num, ratio_den,
                             _ptr(out), _ptr(count), _ptr(ws), ws.numel(), _stream()))
    return out[:nq], count


def match_l2_noalloc(dq, dt, ratio_num: int = 3, ratio_den: int = 4, out=None, count=None):
    """xa_match_l2_noalloc: match_l2 with the library's own per-GPU scratch array in place of a
    workspace.  out / count may be passed in (preallocated), so the call itself allocates
    nothing; calls that overlap on one GPU race on the shared scratch."""
    import torch
    for name, d in (("dq", dq), ("dt", dt)):
        if d.dtype != torch.uint8 or d.dim() != 2 or d.shape[1] != 128 or not d.is_contiguous():
            raise ValueError(f"{name} must be a contiguous uint8 tensor of shape [n, 128]")
    dev = dq.device
    nq, nt = int(dq.shape[0]), int(dt.shape[0])
    if out is None:
        out = torch.empty((max(nq, 1), 3), dtype=torch.int32, device=dev)
    if count is None:
        count = torch.empty(1, dtype=torch.int32, device=dev)
    if out.dtype != torch.int32 or not out.is_contiguous() or out.numel() < 3 * nq:
        raise ValueError("out must be a contiguous int32 tensor of at least n_q x 3 entries")
    _check(lib().xa_match_l2_noalloc(_ptr(dq) if nq else None, nq, _ptr(dt) if nt else None, nt, ratio_num,
                                     ratio_den, _ptr(out), _ptr(count), _stream()))
    return out.view(-1)[:3 * nq].view(nq, 3), count


class SiftOpts(_c.Structure):
    """xa_sift_opts (defaults: 3 layers, sigma0 1.6, input blur 0.5, contrast 0.04, edge 10)."""
    _fields_ = [("n_octaves", _c.c_int32), ("n_layers", _c.c_int32), ("max_keypoints", _c.c_int32),
                ("raw_capacity", _c.c_int32), ("sigma0", _c.c_double), ("sigma_in", _c.c_double),
                ("contrast", _c.c_double), ("edge", _c.c_double)]


def sift_opts(max_keypoints: int = 4096, n_octaves: int = 0, n_layers: int = 3, raw_capacity: int = 0,
              sigma0: float = 1.6, sigma_in: float = 0.5, contrast: float = 0.04, edge: float = 10.0) -> SiftOpts:
    return SiftOpts(n_octaves, n_layers, max_keypoints, raw_capacity, sigma0, sigma_in, contrast, edge)


SIFT_KP_DTYPE = np.dtype([("x", "f4"), ("y", "f4"), ("size", "f4"), ("angle", "f4"), ("response", "f4"),
                          ("xi", "i4"), ("yi", "i4"), ("octave", "i1"), ("layer", "i1"), ("peak", "i1"),
                          ("pad", "i1")])


def extract_sift(img, opts: SiftOpts = None, ws=None):
    """SIFT on a u8 device image [H, W] (xa_extract_sift).  Returns (kp int32 [max, 8] holding
    xa_sift_keypoint records, desc u8 [max, 128], count int32 [2] = written, found); decode the
    keypoints with sift_keypoints_np."""
    import torch
    if img.dtype != torch.uint8 or img.dim() != 2:
        raise ValueError("img must be a uint8 tensor [H, W]")
    if opts is None:
        opts = sift_opts()
    h, w = int(img.shape[0]), int(img.shape[1])
    pitch = int(img.stride(0))
    if img.stride(1) != 1:
        raise ValueError("img rows must be contiguous")
    dev = img.device
    need = lib().xa_sift_workspace_size(w, h, _c.byref(opts))
    if need == 0:
        raise XAError(-1, "invalid SIFT options or image size")
    if ws is None:
        ws = _empty(need, dev)
    m = int(opts.max_keypoints)
    kp = torch.empty((m, 8), dtype=torch.int32, device=dev)
    desc = torch.empty((m, 128), dtype=torch.uint8, device=dev)
    count = torch.empty(2, dtype=torch.int32, device=dev)
    _check(lib().xa_extract_sift(_ptr(img), w, h, pitch, _c.byref(opts), _ptr(kp), _ptr(desc), _ptr(count),
                                 _ptr(ws), ws.numel(), _stream()))
    return kp, desc, count


def sift_keypoints_np(kp, n: int) -> np.ndarray:
    return np.ascontiguousarray(kp[:n].cpu().numpy()).view(SIFT_KP_DTYPE).reshape(-1)


def l2_matches_np(out) -> np.ndarray:
    return np.ascontiguousarray(out.cpu().numpy()).view(L2_MATCH_DTYPE).reshape(-1)


def matches_np(m_tensor) -> np.ndarray:
    a = m_tensor.cpu().numpy()
    return a.reshape(a.shape[0], a.shape[1] * a.shape[2]).view(MATCH_DTYPE)


class StageRunner:
    """Preallocated buffers to run the path stage by stage (simulate, extract, match) for one
    image pair, each stage one C-ABI call on the current stream."""

    def __init__(self, plan_a: Plan, plan_b: Plan, device="cuda"):
        import torch
        self.plan_a, self.plan_b = plan_a, plan_b
        self.device = torch.device(device)
        L = lib()
        z = lambda n, dt=torch.uint8: torch.zeros(max(int(n), 1), dtype=dt, device=self.device)  # noqa: E731
        self.side = {}
        for key, p in (("a", plan_a), ("b", plan_b)):
            N = p.n_features
            self.side[key] = dict(
                plan=p, dev=p.device(self.device), arena=z(p.arena_bytes), mask=z(p.arena_bytes),
                sim_ws=_empty(L.xa_simulate_workspace_size(p.host_ptr()), self.device),
                ext_ws=_empty(L.xa_extract_workspace_size(p.host_ptr()), self.device),
                kp=torch.zeros((p.n_views, N, 40), dtype=torch.uint8, device=self.device),
                desc=torch.zeros((p.n_views, N, 32), dtype=torch.uint8, device=self.device),
                count=torch.zeros(p.n_views, dtype=torch.int32, device=self.device))
        n_pairs = plan_a.n_views * plan_b.n_views
        self.matches = torch.zeros((n_pairs, plan_a.n_features, 8), dtype=torch.uint8, device=self.device)
        self.pair_count = torch.zeros(n_pairs, dtype=torch.int32, device=self.device)
        self.best = torch.zeros(4, dtype=torch.int32, device=self.device)

    def simulate(self, key: str, img):
        s = self.side[key]
        p = s["plan"]
        _check(lib().xa_simulate_views(p.host_ptr(), _ptr(s["dev"]), _ptr(img), _ptr(s["arena"]),
                                       _ptr(s["mask"]), None, _ptr(s["sim_ws"]), s["sim_ws"].numel(), _stream()))

    def extract(self, key: str, pattern):
        s = self.side[key]
        p = s["plan"]
        _check(lib().xa_extract_orb(p.host_ptr(), _ptr(s["dev"]), _ptr(s["arena"]), _ptr(s["mask"]), _ptr(pattern),
                                    _ptr(s["kp"]), _ptr(s["desc"]), _ptr(s["count"]), _ptr(s["ext_ws"]),
                                    s["ext_ws"].numel(), _stream()))

    def match(self, ratio_num: int = 4, ratio_den: int = 5):
        a, b = self.side["a"], self.side["b"]
        _check(lib().xa_match_views(_ptr(a["desc"]), _ptr(a["count"]), self.plan_a.n_views, _ptr(b["desc"]),
                                    _ptr(b["count"]), self.plan_b.n_views, self.plan_a.n_features, ratio_num,
                                    ratio_den, _ptr(self.matches), _ptr(self.pair_count), _ptr(self.best),
                                    _stream()))


# ---------------------------------------------------------------- match plans and batches

GROUP_DTYPE = np.dtype([("a0", "i4"), ("na", "i4"), ("b0", "i4"), ("nb", "i4"), ("pair_base", "i8")])


@dataclass
class MatchPlan:
    blob: np.ndarray
    groups: np.ndarray
    n_features: int
    _dev: object = None

    def host_ptr(self) -> int:
        return self.blob.ctypes.data

    @property
    def total_pairs(self) -> int:
        g = self.groups
        return int((g["pair_base"] + g["na"].astype(np.int64) * g["nb"]).max())

    def device(self, device="cuda"):
        import torch
        if self._dev is None:
            self._dev = torch.from_numpy(self.blob.copy()).to(device)
        return self._dev


def plan_matches(groups, n_features: int, queries_per_lane: int = 0) -> MatchPlan:
    groups = np.ascontiguousarray(groups, GROUP_DTYPE)
    n = ctypes.c_size_t(0)
    _check(lib().xa_plan_matches(groups.ctypes.data, len(groups), n_features, queries_per_lane, None, 0,
                                 ctypes.byref(n)))
    blob = np.zeros(n.value, np.uint8)
    _check(lib().xa_plan_matches(groups.ctypes.data, len(groups), n_features, queries_per_lane, blob.ctypes.data,
                                 blob.size, ctypes.byref(n)))
    return MatchPlan(blob, groups, n_features)


MATCH_MATRIX = -1          # queries_per_lane code of the matrix-core (MFMA) matcher
MATCH_MATRIX_PACKED = -2   # the same with query tiles packed across views
MATCH_VARIANTS = (1, 2, 4, MATCH_MATRIX, MATCH_MATRIX_PACKED)


TUNE_USE_CACHE = 1


def autotune_queries_per_lane(groups, n_features: int, device="cuda", desc=None, count=None, reps: int = 5,
                              use_cache: bool = True, out=None):
    """The matcher variant (the popcount kernel with 1, 2 or 4 queries per lane, or the
    matrix-core kernel, MATCH_MATRIX, plain or with query tiles packed across views,
    MATCH_MATRIX_PACKED) that runs `groups` fastest on this GPU.

    The library's tuner (xa_tune_matcher) times every variant with HIP events on the current
    stream, over the given descriptor set (desc [views][n_features][32], count [views]) or,
    without one, over random descriptors with every view full.  The matcher's work does not
    depend on the descriptor bits but does depend on the counts: uneven counts favour more,
    smaller blocks.  out = (matches, pair_count, best) may bring the result buffers.  The
    library keeps the winner per device, keyed by the group table, n_features and the counts;
    use_cache serves a known key from there, use_cache=False times again.  Returns
    (queries_per_lane, {variant: ms})."""
    import torch
    groups = np.ascontiguousarray(groups, GROUP_DTYPE)
    dev = torch.device(device)
    total = int((groups["pair_base"] + groups["na"].astype(np.int64) * groups["nb"]).max())
    n_views = int(max((groups["a0"] + groups["na"]).max(), (groups["b0"] + groups["nb"]).max()))
    if desc is None:
        gen = torch.Generator(device=dev).manual_seed(1)
        desc = torch.randint(0, 256, (n_views, n_features, 32), dtype=torch.uint8, device=dev, generator=gen)
        count = torch.full((n_views,), n_features, dtype=torch.int32, device=dev)
    if out is None:
        out = (torch.empty((total, n_features, MATCH_DTYPE.itemsize), dtype=torch.uint8, device=dev),
               torch.empty(total, dtype=torch.int32, device=dev),
               torch.empty((len(groups), 4), dtype=torch.int32, device=dev))
    matches, pair_count, best_buf = out
    ws = _empty(lib().xa_tune_matcher_workspace_size(groups.ctypes.data, len(groups), n_features), dev)
    best_q = ctypes.c_int32(0)
    ms = np.zeros(len(MATCH_VARIANTS), np.float32)
    _check(lib().xa_tune_matcher(groups.ctypes.data, len(groups), n_features, _ptr(desc), _ptr(count),
                                 int(desc.shape[0]), reps, TUNE_USE_CACHE if use_cache else 0, _ptr(matches),
                                 _ptr(pair_count), _ptr(best_buf), _ptr(ws), ws.numel(), _stream(),
                                 ctypes.byref(best_q), ms.ctypes.data))
    return int(best_q.value), {q: float(t) for q, t in zip(MATCH_VARIANTS, ms)}

def match_groups(mplan: MatchPlan, desc, count, ratio_num: int = 4, ratio_den: int = 5):
    """Group matching over one descriptor set.  Returns (matches u8[P, N, 8], pair_count i32[P], best i32[G, 4])."""
    import torch
    dev = desc.device
    P, N, G = mplan.total_pairs, mplan.n_features, len(mplan.groups)
    matches = torch.zeros((P, N, 8), dtype=torch.uint8, device=dev)
    pc = torch.zeros(P, dtype=torch.int32, device=dev)
    best = torch.zeros((G, 4), dtype=torch.int32, device=dev)
    _check(lib().xa_match_groups(mplan.host_ptr(), _ptr(mplan.device(dev)), _ptr(desc), _ptr(count), count.numel(),
                                 ratio_num, ratio_den, _ptr(matches), _ptr(pc), _ptr(best), _stream()))
    return matches, pc, best


class BatchRunner:
    """Many image pairs through the batched path.

    One sources buffer holds the originals and the scale-stage outputs; the views of
    consecutive image pairs are grouped into chunks (one view plan each) whose
    simulation and ORB workspace stays under `chunk_bytes`; one match plan has a group
    per image pair.  `pair_views[k]` = (first view of A, n views of A, first view of B,
    n views of B) in the global view numbering.  `ws` may bring a workspace (a uint8
    device tensor of at least `ws_bytes`, 256-byte aligned) shared with other runners
    that are not in flight at the same time, or be set later (allocate_ws=False, then
    set_workspace).  queries_per_lane = "auto" picks the matcher variant with
    autotune_queries_per_lane on the descriptors of the first run or capture."""

    def __init__(self, pairs, grid, scales=(1.0,), n_levels: int = 8, n_features: int = 500,
                 fast_threshold: int = 20, device="cuda", queries_per_lane: int = 0,
                 chunk_bytes: int = 24 << 30, ws=None, allocate_ws: bool = True, interp: str = "lanczos4"):
        import torch
        self.device = torch.device(device)
        L = lib()
        arena = SourceArena()
        jobs, images = [], {}
        # grid rows (t, phi) or (t, phi, s); a structured PARAMS_DTYPE array gives all six parameters
        if isinstance(grid, np.ndarray) and grid.dtype.names:
            rows = [tuple(float(r[k]) for k in ("t", "phi", "psi", "s", "tx", "ty")) for r in grid]
        else:
            rows = [(float(g[0]), float(g[1]), 0.0, float(g[2]) if len(g) > 2 else 1.0, 0.0, 0.0) for g in grid]
        pair_views = []          # per pair: list over sides of [(source index, scale)]
        self.pair_jobs = []      # per pair: its scale-stage jobs
        for (A, B) in pairs:
            sides, pj = [], []
            for img in (A, B):
                si = arena.add(img.shape[1], img.shape[0])
                images[si] = img
                srcs = []
                for sc in scales:
                    if sc == 1.0:
                        srcs.append(si)
                    else:
                        w, h = scaled_size(img.shape[1], img.shape[0], sc)
                        di = arena.add(w, h, sc)
                        jobs.append((arena.descs[si], arena.descs[di], sc))
                        pj.append(jobs[-1])
                        srcs.append(di)
                sides.append(srcs)
            pair_views.append(sides)
            self.pair_jobs.append(pj)
        self.view_rows = rows
        table = arena.table()

        def pair_plan(ps):
            vsrc, params = [], []
            for sides in ps:
                for srcs in sides:
                    for src in srcs:
                        for row in rows:
                            vsrc.append(src)
                            params.append(row)
            return plan_views(table, vsrc, np.array(params, PARAMS_DTYPE), n_levels, 1.2, n_features,
                              fast_threshold, interp), vsrc

        def chunk_ws(plan):
            ptrs = (ctypes.c_void_p * 1)(plan.host_ptr())
            return L.xa_match_batch_workspace_size(None, 1, ptrs)

        # greedy chunks of whole pairs under the workspace budget (a chunk's scratch is the
        # sum of its pairs' scratch: arena, blur and candidate space add up view by view)
        per_pair = [chunk_ws(pair_plan([pv])[0]) for pv in pair_views]
        self.chunks, vsrc_all, cur, cur_bytes = [], [], [], 0
        for k, pv in enumerate(pair_views):
            if cur and cur_bytes + per_pair[k] > chunk_bytes:
                plan0, vs0 = pair_plan(cur)
                self.chunks.append(plan0)
                vsrc_all += vs0
                cur, cur_bytes = [], 0
            cur.append(pv)
            cur_bytes += per_pair[k]
        if cur:
            plan0, vs0 = pair_plan(cur)
            self.chunks.append(plan0)
            vsrc_all += vs0
        nvs = len(rows) * len(scales)
        groups, self.pair_views, base, v = [], [], 0, 0
        for _ in pairs:
            a0, b0 = v, v + nvs
            groups.append((a0, nvs, b0, nvs, base))
            self.pair_views.append((a0, nvs, b0, nvs))
            base += nvs * nvs
            v += 2 * nvs
        self.arena = arena
        self.splan = plan_scales(np.array(jobs, SCALE_JOB_DTYPE)) if jobs else None
        self.autotune = None
        self._tune = queries_per_lane == "auto"
        self.mplan = plan_matches(np.array(groups, GROUP_DTYPE), n_features, 0 if self._tune else queries_per_lane)
        self.mplan_q = int(np.frombuffer(self.mplan.blob, np.int32, 4)[3])
        self.view_scale = np.array([arena.descs[s][5] for s in vsrc_all])
        self.view_source = list(vsrc_all)     # source index of each view (global numbering)
        self.n_views = len(vsrc_all)
        dev = self.device
        self.sources = torch.from_numpy(arena.pack(images)).to(dev)
        nv, N = self.n_views, n_features
        z = lambda *sh, dt=torch.uint8: torch.zeros(sh, dtype=dt, device=dev)  # noqa: E731
        self.kp, self.desc, self.count = z(nv, N, 40), z(nv, N, 32), z(nv, dt=torch.int32)
        P = self.mplan.total_pairs
        self.matches, self.pair_count = z(P, N, 8), z(P, dt=torch.int32)
        self.best = z(len(groups), 4, dt=torch.int32)
        nc = len(self.chunks)
        self._hosts = (ctypes.c_void_p * nc)(*[c.host_ptr() for c in self.chunks])
        self._devs = (ctypes.c_void_p * nc)(*[_ptr(c.device(dev)) for c in self.chunks])
        sp = self.splan.host_ptr() if self.splan else None
        need = L.xa_match_batch_workspace_size(sp, nc, self._hosts)
        if need == 0:
            raise XAError(-1, "invalid batch plans")
        self.ws_bytes = need
        if ws is not None and ws.numel() < need:
            raise XAError(-2, f"batch workspace needs {need} bytes, got {ws.numel()}")
        self.ws = ws if ws is not None else (_empty(need, dev) if allocate_ws else None)
        self.bufs = _BatchBuffers(*[_ptr(t) for t in (self.kp, self.desc, self.count, self.matches,
                                                      self.pair_count, self.best)])
        self.graph = None

    def precision(self, k: int, H, th: float = 2.0, ratio_num: int = 4, ratio_den: int = 5):
        """Eqs. (5)-(6) on pair k's best view pair: device int32 [correct, accepted]."""
        import torch
        a0, na, b0, nb = self.pair_views[k]
        base = int(self.mplan.groups[k]["pair_base"])
        N = self.mplan.n_features
        out = torch.zeros(2, dtype=torch.int32, device=self.device)
        Hc = np.ascontiguousarray(H, np.float64).reshape(9)
        _check(lib().xa_pair_precision(_ptr(self.kp[a0]), _ptr(self.kp[b0]), _ptr(self.matches[base]),
                                       _ptr(self.count[a0:]), _ptr(self.count[b0:]), nb, N, ratio_num, ratio_den,
                                       _ptr(self.best[k]), Hc.ctypes.data, th, _ptr(out), _stream()))
        return out

    def set_workspace(self, ws):
        """Use `ws` (uint8 device tensor of at least ws_bytes) from now on."""
        if ws.numel() < self.ws_bytes:
            raise XAError(-2, f"batch workspace needs {self.ws_bytes} bytes, got {ws.numel()}")
        self.close()
        self.ws = ws

    def _call_args(self):
        if self.ws is None:
            raise XAError(-1, "no workspace: pass ws or call set_workspace")
        sp = self.splan.host_ptr() if self.splan else None
        sd = _ptr(self.splan.device(self.device)) if self.splan else None
        return (sp, sd, len(self.chunks), self._hosts, self._devs, self.mplan.host_ptr(),
                _ptr(self.mplan.device(self.device)), _ptr(self.sources))

    def _tune_matcher(self, pattern, ratio_num, ratio_den):
        """First run with queries_per_lane = "auto": run once, time the matcher variants on the
        descriptor sets this batch produced, and re-plan the matcher with the fastest."""
        self._tune = False
        self.run(pattern, ratio_num, ratio_den)
        q, ms = autotune_queries_per_lane(self.mplan.groups, self.mplan.n_features, self.device, self.desc, self.count,
                                          out=(self.matches, self.pair_count, self.best))
        self.autotune = {"queries_per_lane": q, "ms": ms}
        if q != self.mplan_q:
            self.close()
            self.mplan = plan_matches(self.mplan.groups, self.mplan.n_features, q)
            self.mplan_q = q

    def run(self, pattern, ratio_num: int = 4, ratio_den: int = 5):
        if self._tune:
            self._tune_matcher(pattern, ratio_num, ratio_den)
        _check(lib().xa_match_batch(*self._call_args(), _ptr(pattern), ratio_num, ratio_den, ctypes.byref(self.bufs),
                                    _ptr(self.ws), self.ws.numel(), _stream()))

    def capture(self, pattern, ratio_num: int = 4, ratio_den: int = 5):
        if self._tune:
            self._tune_matcher(pattern, ratio_num, ratio_den)
        self.close()
        g = ctypes.c_void_p(0)
        _check(lib().xa_match_batch_capture(*self._call_args(), _ptr(pattern), ratio_num, ratio_den,
                                            ctypes.byref(self.bufs), _ptr(self.ws), self.ws.numel(), ctypes.byref(g)))
        self.graph = g
        self._pattern = pattern       # the graph reads this buffer on every replay

    def replay(self):
        if not self.graph:
            raise XAError(-1, "no captured graph")
        _check(lib().xa_graph_launch(self.graph, _stream()))

    def close(self):
        if self.graph:
            lib().xa_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- differentiable warp

def _check_crops(img, params):
    import torch
    if img.dtype != torch.float32 or img.dim() != 3 or not img.is_contiguous():
        raise XAError(-1, "img must be a contiguous float32 tensor [n, h, w]")
    if params.dtype != torch.float64 or tuple(params.shape) != (img.shape[0], 6) or not params.is_contiguous():
        raise XAError(-1, "params must be a contiguous float64 tensor [n, 6] (t, phi, psi, s, tx, ty)")
    if params.device != img.device:
        raise XAError(-1, "img and params must be on the same device")


def warp_f32_fwd(img, params):
    """(out [n, h, w] fp32, mask [n, h, w] u8) for crops img [n, h, w] and params [n, 6] fp64."""
    import torch
    _check_crops(img, params)
    n, h, w = img.shape
    out = torch.empty_like(img)
    mask = torch.empty((n, h, w), dtype=torch.uint8, device=img.device)
    ws = _empty(lib().xa_warp_f32_fwd_workspace_size(n, h, w), img.device)
    _check(lib().xa_warp_f32_fwd(_ptr(img), n, h, w, _ptr(params), _ptr(out), _ptr(mask), _ptr(ws), ws.numel(),
                                 _stream()))
    return out, mask


def warp_f32_bwd(img, gout, params, need_img: bool = True, need_params: bool = True):
    """(d/dimg [n, h, w] fp32 or None, d/dparams [n, 6] fp64 or None) for dLoss/dout = gout."""
    import torch
    _check_crops(img, params)
    gout = gout.contiguous()
    if gout.shape != img.shape or gout.dtype != torch.float32:
        raise XAError(-1, "gout must be float32 with the shape of img")
    n, h, w = img.shape
    gimg = torch.empty_like(img) if need_img else None
    gpar = torch.empty((n, 6), dtype=torch.float64, device=img.device) if need_params else None
    ws = _empty(lib().xa_warp_f32_bwd_workspace_size(n, h, w), img.device)
    _check(lib().xa_warp_f32_bwd(_ptr(img), _ptr(gout), _ptr(params), n, h, w, _ptr(gimg), _ptr(gpar), _ptr(ws),
                                 ws.numel(), _stream()))
    return gimg, gpar


def _warp_function():
    import torch

    class WarpF32(torch.autograd.Function):
        """Lanczos-4 affine warp of fp32 crops; differentiable in the crops and the
        six camera parameters (forward and adjoint are the library's kernels)."""

        @staticmethod
        def forward(ctx, img, params):
            out, mask = warp_f32_fwd(img, params)
            ctx.save_for_backward(img, params)
            ctx.mark_non_differentiable(mask)
            return out, mask

        @staticmethod
        def backward(ctx, gout, _gmask):
            img, params = ctx.saved_tensors
            gi, gp = warp_f32_bwd(img, gout, params, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
            return gi, gp

    return WarpF32


_WARP_FN = None


def warp_f32(img, params):
    """Differentiable warp: returns (out, mask); gradients flow to img and params."""
    global _WARP_FN
    if _WARP_FN is None:
        _WARP_FN = _warp_function()
    return _WARP_FN.apply(img.contiguous(), params.contiguous())


def blur_f32(x, sigma: float):
    """Separable Gaussian (replicated border, |k| <= ceil(3 sigma)) of fp32 crops [n, h, w] by
    xa_blur_f32; sigma 0 returns x."""
    import torch
    if sigma <= 0:
        return x
    x = x.contiguous()
    if x.dtype != torch.float32 or x.dim() != 3:
        raise XAError(-1, "need float32 crops [n, h, w]")
    n, h, w = x.shape
    out = torch.empty_like(x)
    ws = _empty(lib().xa_blur_f32_workspace_size(n, h, w), x.device)
    _check(lib().xa_blur_f32(_ptr(x), n, h, w, float(sigma), _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def refine_tilt(img, target, params, grid, target_mask=None, steps: int = 20, lr: float = 0.03, sigmas=None):
    """Photometric refinement of (t, phi) for each crop.

    The grid search comes first: every (t, phi) of `grid` is warped (one batched
    forward per grid point) and the one with the lowest mean squared error over the
    pixels valid in both the warped crop and the target is kept.  Then `steps` Adam
    steps on (log t, phi) start from it, coarse to fine (crop and target smoothed by a
    Gaussian of sigma 4 px for the first half of the steps and 1 px for the rest,
    unless `sigmas` gives one sigma per step), with the other four parameters held.
    The grid point decides: a crop keeps its refined (t, phi) only if the refined loss on
    the unsmoothed crops is lower.
    Returns (params [n, 6], grid_loss [n], refined_loss [n])."""
    import torch
    n = img.shape[0]
    base = params.detach().clone()
    tmask = torch.ones_like(target) if target_mask is None else target_mask.to(target.dtype)
    if sigmas is None:
        sigmas = [4.0] * (steps // 2) + [1.0] * (steps - steps // 2)
    if len(sigmas) != steps:
        raise XAError(-1, "need one sigma per step")

    def losses(im, tg, p):
        out, mask = warp_f32(im, p)
        m = mask.to(im.dtype) * tmask
        r = (out - tg) * m
        return (r * r).sum(dim=(1, 2)) / m.sum(dim=(1, 2)).clamp_min(1.0)

    with torch.no_grad():
        best = torch.full((n,), float("inf"), dtype=torch.float64, device=img.device)
        best_p = base.clone()
        for (t, phi) in grid:
            p = base.clone()
            p[:, 0] = t
            p[:, 1] = phi
            l = losses(img, target, p).double()
            better = l < best
            best = torch.where(better, l, best)
            best_p[better] = p[better]
    logt = best_p[:, 0].log().clone().requires_grad_(True)
    phi = best_p[:, 1].clone().requires_grad_(True)
    opt = torch.optim.Adam([logt, phi], lr=lr)
    smoothed = {}
    for sg in sigmas:
        if sg not in smoothed:
            smoothed[sg] = (blur_f32(img, sg), blur_f32((target * tmask).contiguous(), sg))
        im, tg = smoothed[sg]
        opt.zero_grad()
        p = torch.cat([logt.exp()[:, None], phi[:, None], best_p[:, 2:]], dim=1)
        losses(im, tg, p).sum().backward()
        opt.step()
    with torch.no_grad():
        p = torch.cat([logt.exp()[:, None], phi[:, None], best_p[:, 2:]], dim=1)
        refined = losses(img, target, p).double()
        keep = refined < best
        out = torch.where(keep[:, None], p, best_p)
    return out, best, refined


# ---------------------------------------------------------------- precise stage

def ransac_homography(pa, pb, samples, th: float = 3.0):
    """Homography RANSAC (device tensors pa, pb [n, 2] fp64, samples [k, 4] int32).
    Returns (scores [k] i32, best [2] i32, H [3, 3] f64, inliers [n] u8), all on the device."""
    import torch
    dev = pa.device
    n, k = int(pa.shape[0]), int(samples.shape[0])
    scores = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
    best = torch.empty(2, dtype=torch.int32, device=dev)
    H = torch.empty(9, dtype=torch.float64, device=dev)
    inl = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    _check(lib().xa_ransac_homography(_ptr(pa.contiguous()), _ptr(pb.contiguous()), n, _ptr(samples.contiguous()), k,
                                      th, _ptr(scores), _ptr(best), _ptr(H), _ptr(inl), _stream()))
    return scores[:k], best, H.view(3, 3), inl[:n]


def best_pair_points(kp_a, kp_b, matches, count_a, count_b, best, n_b: int, n_features: int,
                     ratio_num: int = 4, ratio_den: int = 5):
    """Accepted matches of the best view pair as original-image points: (pa, pb, dist, n) on the
    device, pa/pb/dist of capacity n_features (dist = Hamming distances)."""
    import torch
    dev = kp_a.device
    pa = torch.empty((n_features, 2), dtype=torch.float64, device=dev)
    pb = torch.empty((n_features, 2), dtype=torch.float64, device=dev)
    dist = torch.empty(n_features, dtype=torch.int32, device=dev)
    n = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().xa_best_pair_points(_ptr(kp_a), _ptr(kp_b), _ptr(matches), _ptr(count_a), _ptr(count_b), n_b,
                                     n_features, ratio_num, ratio_den, _ptr(best), _ptr(pa), _ptr(pb), _ptr(dist),
                                     _ptr(n), _stream()))
    return pa, pb, dist, n


def draw_samples(n: int, k: int, seed: int = 0) -> np.ndarray:
    """k RANSAC samples of 4 distinct match indices out of n (host numpy, seeded PCG64)."""
    g = np.random.Generator(np.random.PCG64(seed))
    if n < 4:
        return np.zeros((0, 4), np.int32)
    return np.stack([g.choice(n, 4, replace=False) for _ in range(k)]).astype(np.int32)


def sift_features(img, opts: "SiftOpts" = None):
    """SIFT keypoints and descriptors of a u8 device image: (kp, desc, n) with n the host count
    (one synchronisation: the L2 matcher takes its sizes on the host)."""
    kp, desc, count = extract_sift(img, opts)
    n = int(count[0].item())
    return kp, desc, n


def sift_match_points(fq, ft, ratio_num: int = 3, ratio_den: int = 4, map_q=None, map_t=None):
    """L2 matching of the query features fq against the train features ft (xa_match_l2) and the
    kept matches' points and distances (xa_sift_match_points): (pq, pt, des, n) on the device,
    points taken through the 2 x 3 maps map_q / map_t (None = identity)."""
    import torch
    kq, dq, nq = fq
    kt, dt, nt = ft
    dev = kq.device
    out, _ = match_l2(dq[:nq], dt[:nt], ratio_num, ratio_den)
    pq = torch.empty((max(nq, 1), 2), dtype=torch.float64, device=dev)
    pt = torch.empty((max(nq, 1), 2), dtype=torch.float64, device=dev)
    des = torch.empty(max(nq, 1), dtype=torch.float64, device=dev)
    n = torch.empty(1, dtype=torch.int32, device=dev)
    mq = None if map_q is None else np.ascontiguousarray(map_q, np.float64).reshape(6)
    mt = None if map_t is None else np.ascontiguousarray(map_t, np.float64).reshape(6)
    _check(lib().xa_sift_match_points(_ptr(kq), _ptr(kt), _ptr(out), nq, nt, ratio_num, ratio_den,
                                      None if mq is None else mq.ctypes.data, None if mt is None else mt.ctypes.data,
                                      _ptr(pq), _ptr(pt), _ptr(des), _ptr(n), _stream()))
    return pq, pt, des, n


def simulated_view(img, params, interp: str = "lanczos4"):
    """One simulated view of a u8 device image (the camera change of eq. (2), Lanczos-4 of
    eqs. (3)-(4) after the anti-alias blur): (view u8 [H', W'] device tensor (a strided view
    into the arena), inverse map view -> image as 6 floats)."""
    plan = plan_image(int(img.shape[1]), int(img.shape[0]), make_params([tuple(params)]), 1, 1.2, 1, 20,
                      interp=interp)
    arena, _ = simulate_views(plan, img.contiguous())
    v = plan.views[0]
    o, w, h, p = int(v["offset"]), int(v["width"]), int(v["height"]), int(v["pitch"])
    return arena[o:o + p * h].view(h, p)[:, :w], np.array(v["inv"], np.float64)


def precise_stage(A, B, params_a, params_b, opts: "SiftOpts" = None, ransac_k: int = 2000, th: float = 3.0,
                  seed: int = 0, ratio_num: int = 3, ratio_den: int = 4):
    """The stage after the search (Sec. III.C): A and B (device u8 originals) are re-simulated
    with Lanczos-4 at the best parameters (xa_affine_params rows), SIFT runs on both views, the
    views' L2 matches (ratio num/den, Sec. IV.C) are taken back to the original images through the
    views' inverse maps and screened by homography RANSAC; eq. (7) gives the inlier share.
    Returns a dict with H (3x3 numpy, A original -> B original), the number of matches, of
    inliers and their ratio, and the device point/inlier arrays."""
    import torch
    va, inv_a = simulated_view(A, params_a)
    vb, inv_b = simulated_view(B, params_b)
    fa, fb = sift_features(va, opts), sift_features(vb, opts)
    pa, pb, _, n_dev = sift_match_points(fa, fb, ratio_num, ratio_den, inv_a, inv_b)
    n = int(n_dev.item())
    samples = torch.from_numpy(draw_samples(n, ransac_k, seed)).to(A.device)
    scores, best, H, inl = ransac_homography(pa[:n], pb[:n], samples, th)
    n_in = int(best[1].item())
    return {"H": H.cpu().numpy(), "matches": n, "inliers": max(n_in, 0),
            "inlier_ratio": max(n_in, 0) / n if n > 0 else 0.0, "pa": pa[:n], "pb": pb[:n], "inlier_mask": inl,
            "samples": samples, "scores": scores, "keypoints": (fa[2], fb[2])}


def scaling_coefficient(pa, pb, dist, n):
    """Eq. (1) on device points/distances (as from best_pair_points); returns a device fp64 [1]."""
    import torch
    f = torch.empty(1, dtype=torch.float64, device=pa.device)
    _check(lib().xa_scaling_coefficient(_ptr(pa), _ptr(pb), _ptr(dist), _ptr(n), int(pa.shape[0]), _ptr(f),
                                        _stream()))
    return f


def scaling_coefficient_f64(pa, pb, des, n):
    """Eq. (1) with fp64 descriptor distances (xa_scaling_coefficient_f64); a device fp64 [1]."""
    import torch
    f = torch.empty(1, dtype=torch.float64, device=pa.device)
    _check(lib().xa_scaling_coefficient_f64(_ptr(pa), _ptr(pb), _ptr(des), _ptr(n), int(pa.shape[0]), _ptr(f),
                                            _stream()))
    return f


def select_base_image(A, B, opts: "SiftOpts" = None, ratio_num: int = 3, ratio_den: int = 4):
    """Base-image selection of Sec. III.A on the unsimulated images: SIFT on A and B, L2 matching
    A -> B gives f1 and B -> A gives f2 by eq. (1) over the kept matches in query order, with
    their SIFT descriptor distances; A is the base when f1 > f2.  Returns ("A" | "B", f1, f2)."""
    fa, fb = sift_features(A, opts), sift_features(B, opts)
    f = []
    for fq, ft in ((fa, fb), (fb, fa)):
        pq, pt, des, n = sift_match_points(fq, ft, ratio_num, ratio_den)
        f.append(float(scaling_coefficient_f64(pq, pt, des, n).item()))
    return ("A" if f[0] > f[1] else "B"), f[0], f[1]
