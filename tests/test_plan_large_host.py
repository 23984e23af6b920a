"""Host-only: the plan of the large-view stress pair (564 views of sources 712 x 3072 and
4096 x 534 at scales 1, 0.5, 0.25; 8 levels, 2000 keypoints) lays out its pyramid arena, candidate
arena and blurred planes as disjoint regions inside the sizes it reports, with 64-bit offsets:
its batch workspace is larger than 2^31 bytes, so a 32-bit offset anywhere would overlap or
wrap.  No device work."""
import ctypes
import math
import os

import numpy as np
import pytest

X = pytest.importorskip("paper_2503_03479_amd.xaffine")

T80 = 1.0 / math.cos(math.radians(80.0))


@pytest.fixture(scope="module")
def stress_plan():
    if not os.path.exists(X.LIB_PATH):
        pytest.skip("libxaffine.so not built")
    sizes = [(int(math.ceil(4096 / T80 - 1e-7)), 3072), (4096, int(math.ceil(3072 / T80 - 1e-7)))]
    assert sizes == [(712, 3072), (4096, 534)]
    grid = X.sampling_grid(7)
    rows = [(float(r["t"]), float(r["phi"]), 0.0, 1.0, 0.0, 0.0) for r in grid]
    arena, jobs, vsrc, params = X.SourceArena(), [], [], []
    for (w, h) in sizes:
        si = arena.add(w, h)
        for s in (1.0, 0.5, 0.25):
            src = si
            if s != 1.0:
                ws, hs = X.scaled_size(w, h, s)
                src = arena.add(ws, hs, s)
                jobs.append((arena.descs[si], arena.descs[src], s))
            vsrc += [src] * len(rows)
            params += rows
    plan = X.plan_views(arena.table(), vsrc, np.array(params, X.PARAMS_DTYPE), 8, 1.2, 2000, 20)
    splan = X.plan_scales(np.array(jobs, X.SCALE_JOB_DTYPE))
    return plan, splan


def _disjoint(starts, lengths, total):
    keep = lengths > 0
    s, n = starts[keep].astype(np.int64), lengths[keep].astype(np.int64)
    order = np.argsort(s, kind="stable")
    s, e = s[order], s[order] + n[order]
    return bool(s.min(initial=0) >= 0 and e.max(initial=0) <= total and np.all(e[:-1] <= s[1:]))


def test_stress_plan_sizes(stress_plan):
    plan, splan = stress_plan
    assert plan.n_views == 564 and plan.n_levels == 8
    ptrs = (ctypes.c_void_p * 1)(plan.host_ptr())
    ws = X.lib().xa_match_batch_workspace_size(splan.host_ptr(), 1, ptrs)
    assert ws > 2 ** 31, ws


def test_stress_plan_pyramid_regions_are_disjoint(stress_plan):
    plan, _ = stress_plan
    lv = plan.levels
    assert np.all(lv["pitch"] >= lv["width"])
    lengths = lv["pitch"].astype(np.int64) * lv["height"]
    assert _disjoint(lv["offset"], lengths, plan.arena_bytes)
    v0 = lv.reshape(plan.n_views, plan.n_levels)[:, 0]
    assert np.array_equal(v0["offset"], plan.views["offset"])


def test_stress_plan_candidate_regions_are_disjoint(stress_plan):
    plan, _ = stress_plan
    lv = plan.levels
    h = np.frombuffer(plan.blob, X.HEADER_DTYPE, 1)[0]
    cap = lv["cand_cap"]
    full = ((lv["width"].astype(np.int64) + 1) // 2) * ((lv["height"].astype(np.int64) + 1) // 2)
    assert np.all((cap == 0) | (cap == full))
    assert _disjoint(lv["cand_offset"], cap, int(h["cand_total"]))


def test_stress_plan_blur_planes_are_disjoint(stress_plan):
    plan, _ = stress_plan
    v = plan.views
    h = np.frombuffer(plan.blob, X.HEADER_DTYPE, 1)[0]
    blurred = v["blur_offset"] >= 0
    assert np.array_equal(blurred, v["sigma"] > 0)
    n_tilted = int((X.sampling_grid(7)["t"] > 1.0).sum())
    assert blurred.sum() == 2 * 3 * n_tilted     # every view with t > 1, on each of the 6 sources
    lengths = np.where(blurred, (v["src_w"].astype(np.int64) + 3) // 4 * 4 * v["src_h"], 0)
    assert _disjoint(np.where(blurred, v["blur_offset"], 0), lengths, int(h["blur_floats"]))
