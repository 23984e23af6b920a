"""Host-side checks of libxaffine: exports, the planner against the oracle, argument errors.

No GPU work is launched here; the planner and the argument checks run on the host."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import plan as OP
from oracle import simulate as OS

X = pytest.importorskip("paper_2503_03479_amd.xaffine")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(X.LIB_PATH):
        pytest.skip("libxaffine.so not built")
    return X.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "xaffine.h")).read()
    declared = set(re.findall(r"\b(xa_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(X.EXPORTS)


def test_sampling_grid_equals_oracle(L):
    for n in range(0, 8):
        got = X.sampling_grid(n)
        ref = OP.sampling_grid(n)
        assert len(got) == len(ref)
        assert np.array_equal(got["t"], [t for t, _ in ref])
        assert np.array_equal(got["phi"], [f for _, f in ref])
    assert len(X.sampling_grid(5)) == 45


@pytest.mark.parametrize("w,h,n_tilt", [(256, 256, 2), (1024, 768, 5), (239, 286, 2), (97, 53, 7)])
def test_plan_matches_oracle(L, w, h, n_tilt):
    grid = OP.sampling_grid(n_tilt)
    rows = [(t, f, 0.0, 1.0) for t, f in grid] + [(1.7, 0.4, 0.3, 1.4), (2.5, 2.9, -1.2, 1.3), (3.0, 1.1, 0.2, 4.0)]
    params = X.make_params(rows)
    N, Lv = 1000, 8
    p = X.plan_image(w, h, params, Lv, 1.2, N, 20)
    quotas = OP.level_quotas(N, Lv)
    for i, r in enumerate(rows):
        v = OP.plan_view(w, h, *r)
        pv = p.views[i]
        assert (pv["width"], pv["height"]) == (v.width, v.height)
        assert np.allclose(pv["fwd"].reshape(2, 3), v.fwd, rtol=0, atol=1e-10)
        assert np.allclose(pv["inv"].reshape(2, 3), v.inv, rtol=0, atol=1e-9)
        assert pv["sigma"] == pytest.approx(v.sigma, abs=1e-15)
        assert (pv["ux"], pv["uy"]) == pytest.approx(v.u, abs=1e-16)
        dims = OP.level_dims(v.width, v.height, Lv)
        assert [(int(a), int(b)) for a, b in zip(p.levels[i]["width"], p.levels[i]["height"])] == dims
        assert p.levels[i]["quota"].tolist() == quotas
        assert p.levels[i]["kp_base"].tolist() == [sum(quotas[:l]) for l in range(Lv)]
        if v.sigma > 0:
            major, m, ks, g = OS.blur_taps(v.sigma, v.u)
            assert pv["blur_major"] == major and pv["blur_ntaps"] == len(ks)
            taps = p.taps()[pv["blur_tap0"]:pv["blur_tap0"] + pv["blur_ntaps"]]
            assert np.array_equal(taps["dmaj"], ks)
            km = ks * m
            f = km - np.floor(km)
            assert np.array_equal(taps["dmin"], np.floor(km).astype(np.int64))
            assert np.allclose(taps["wa"], g * (1 - f), rtol=1e-6, atol=1e-9)
            assert np.allclose(taps["wb"], g * f, rtol=1e-6, atol=1e-9)
        else:
            assert pv["blur_ntaps"] == 0 and pv["blur_offset"] == -1
    # arena layout: levels do not overlap and fit the arena
    ends = []
    for lv in p.levels.reshape(-1):
        assert lv["pitch"] >= lv["width"] and lv["pitch"] % 16 == 0 and lv["offset"] % 128 == 0
        ends.append((int(lv["offset"]), int(lv["offset"]) + int(lv["pitch"]) * int(lv["height"])))
    ends.sort()
    assert all(a[1] <= b[0] for a, b in zip(ends, ends[1:]))
    assert ends[-1][1] <= p.arena_bytes


def test_plan_rejects_bad_arguments(L):
    good = X.make_params([(1.0, 0.0)])
    for rows in ([(0.5, 0.0)], [(1.0, 0.0, 0.0, 0.0)], [(1.0, 0.0, 0.0, 0.5)], [(float("nan"), 0.0)],
                 [(2.0, float("inf"))]):
        with pytest.raises(X.XAError) as e:
            X.plan_image(64, 64, X.make_params(rows))
        assert e.value.status == X.XA_EINVAL
    with pytest.raises(X.XAError) as e:
        X.plan_image(0, 64, good)
    assert e.value.status == X.XA_EINVAL
    with pytest.raises(X.XAError) as e:
        X.plan_image(64, 64, good, n_levels=0)
    assert e.value.status == X.XA_EINVAL
    with pytest.raises(X.XAError) as e:
        X.plan_image(64, 64, good, n_features=5000)
    assert e.value.status == X.XA_EUNSUPPORTED
    with pytest.raises(X.XAError) as e:
        X.plan_image(64, 64, good, fast_threshold=300)
    assert e.value.status == X.XA_EINVAL


def test_grid_capacity_error(L):
    import ctypes
    n = ctypes.c_int32(0)
    buf = np.zeros(3, X.PARAMS_DTYPE)
    st = L.xa_sampling_grid(5, 72.0, buf.ctypes.data, 3, ctypes.byref(n))
    assert st == X.XA_ECAPACITY and n.value == 45
    assert b"capacity" in L.xa_last_error()
    assert L.xa_sampling_grid(-1, 72.0, None, 0, ctypes.byref(n)) == X.XA_EINVAL


def test_workspace_queries_and_bad_plan(L):
    p = X.plan_image(128, 96, X.sampling_grid(2), 3, 1.2, 300, 20)
    assert L.xa_simulate_workspace_size(p.host_ptr()) == 4 * 9 * 128 * 96    # nine blurred views
    assert L.xa_extract_workspace_size(p.host_ptr()) > p.arena_bytes
    assert L.xa_match_pair_workspace_size(p.host_ptr(), p.host_ptr()) > 4 * p.arena_bytes
    junk = np.zeros(256, np.uint8)
    assert L.xa_simulate_workspace_size(junk.ctypes.data) == 0
    st = L.xa_simulate_views(junk.ctypes.data, None, None, None, None, None, None, 0, None)
    assert st == X.XA_EINVAL


def test_device_calls_validate_before_launch(L):
    """Argument errors are reported on the host, before anything is enqueued."""
    p = X.plan_image(64, 64, X.sampling_grid(1), 2, 1.2, 100, 20)
    hp = p.host_ptr()
    # NULL device pointers
    assert L.xa_simulate_views(hp, hp, None, None, None, None, None, 0, None) == X.XA_EINVAL
    # too-small workspace (non-NULL dummy pointers are never dereferenced on the host)
    st = L.xa_extract_orb(hp, hp, 256, 256, 256, 256, 256, 256, 256, 0, None)
    assert st == X.XA_ECAPACITY
    assert L.xa_match_views(256, 256, 0, 256, 256, 1, 100, 4, 5, 256, 256, 256, None) == X.XA_EINVAL
    assert L.xa_match_views(256, 256, 1, 256, 256, 1, 100, 4, 0, 256, 256, 256, None) == X.XA_EINVAL
    # the two simulate stages: NULL pointers, a short workspace, a blob that is not a plan
    assert L.xa_blur_views(hp, hp, None, 256, 1 << 30, None) == X.XA_EINVAL
    assert L.xa_blur_views(hp, hp, 256, 256, 0, None) == X.XA_ECAPACITY
    assert L.xa_warp_views(hp, hp, 256, None, 256, None, 256, 1 << 30, None) == X.XA_EINVAL
    assert L.xa_warp_views(hp, hp, 256, 256, 256, None, 256, 0, None) == X.XA_ECAPACITY
    junk = np.zeros(256, np.uint8)
    assert L.xa_warp_views(junk.ctypes.data, hp, 256, 256, 256, None, 256, 1 << 30, None) == X.XA_EINVAL
    # the L2 matcher: counts, ratio, NULL, misaligned and short-workspace arguments
    need = L.xa_match_l2_workspace_size(1000, 700)
    assert need > 0 and L.xa_match_l2_workspace_size(0, 700) == 0 and L.xa_match_l2_workspace_size(-1, 5) == 0
    assert L.xa_match_l2(256, -1, 256, 5, 3, 4, 256, 256, 256, need, None) == X.XA_EINVAL
    assert L.xa_match_l2(256, 5, 256, (1 << 20) + 1, 3, 4, 256, 256, 256, need, None) == X.XA_EINVAL
    assert L.xa_match_l2(256, 1000, 256, 700, 3, 0, 256, 256, 256, need, None) == X.XA_EINVAL
    assert L.xa_match_l2(None, 1000, 256, 700, 3, 4, 256, 256, 256, need, None) == X.XA_EINVAL
    assert L.xa_match_l2(256, 1000, 256, 700, 3, 4, 256, None, 256, need, None) == X.XA_EINVAL
    assert L.xa_match_l2(264, 1000, 256, 700, 3, 4, 256, 256, 256, need, None) == X.XA_EINVAL
    assert L.xa_match_l2(256, 1000, 256, 700, 3, 4, 256, 256, 256, need - 16, None) == X.XA_EINVAL


def test_match_plan_rules():
    G = X.GROUP_DTYPE
    mp = X.plan_matches(np.array([(0, 3, 3, 4, 0), (7, 2, 0, 2, 12)], G), 500)
    assert mp.total_pairs == 16
    with pytest.raises(X.XAError):          # overlapping pair ranges
        X.plan_matches(np.array([(0, 3, 3, 4, 0), (7, 2, 0, 2, 11)], G), 500)
    with pytest.raises(X.XAError):          # negative field
        X.plan_matches(np.array([(0, -1, 3, 4, 0)], G), 500)
    with pytest.raises(X.XAError):          # bad variant
        X.plan_matches(np.array([(0, 1, 1, 1, 0)], G), 500, 3)
    with pytest.raises(X.XAError):          # n_features out of range
        X.plan_matches(np.array([(0, 1, 1, 1, 0)], G), 0)
    # empty groups may share a pair_base
    X.plan_matches(np.array([(0, 0, 3, 4, 0), (7, 2, 0, 2, 0)], G), 500)


def test_match_groups_rejects_views_outside_the_set():
    mp = X.plan_matches(np.array([(0, 3, 3, 4, 0)], X.GROUP_DTYPE), 64)
    fake = ctypes.c_void_p(256)               # never dereferenced: the check comes first
    st = X.lib().xa_match_groups(mp.host_ptr(), fake, fake, fake, 6, 4, 5, fake, fake, fake, None)
    assert st == -1 and b"views" in X.lib().xa_last_error()


def test_batch_chunking_on_host():
    """BatchRunner's planning (no device work): views are numbered pair by pair, each
    pair is one match group, and a small budget splits the views into one chunk per pair
    whose workspace is the largest pair's."""
    import synth
    torch = pytest.importorskip("torch")
    pairs = [synth.make_pair(w, h, 10, 8, seed, 1.5, 0.0, 0.3, supersample=1)
             for (w, h, seed) in ((96, 80, 1), (120, 64, 2), (64, 64, 3))]
    imgs = [(p.A, np.ascontiguousarray(p.B)) for p in pairs]
    grid = [(t, f) for t, f in OP.sampling_grid(1)]
    one = X.BatchRunner(imgs, grid, (1.0, 0.5), n_levels=2, n_features=64, device="cpu")
    many = X.BatchRunner(imgs, grid, (1.0, 0.5), n_levels=2, n_features=64, device="cpu", chunk_bytes=1)
    nvs = 2 * len(grid)
    assert len(one.chunks) == 1 and len(many.chunks) == 3
    assert one.n_views == many.n_views == 3 * 2 * nvs
    assert sum(c.n_views for c in many.chunks) == many.n_views
    assert [tuple(g)[:4] for g in many.mplan.groups] == [(2 * k * nvs, nvs, (2 * k + 1) * nvs, nvs) for k in range(3)]
    assert many.mplan.total_pairs == 3 * nvs * nvs
    per = [X.lib().xa_match_batch_workspace_size(None, 1, (ctypes.c_void_p * 1)(c.host_ptr())) for c in many.chunks]
    # each scratch region is sized for its largest chunk, so the total is at most the sum of those maxima
    assert many.ws.numel() <= 1.25 * (max(per) + X.lib().xa_scale_workspace_size(many.splan.host_ptr()))
    assert many.ws.numel() < one.ws.numel()
    # scale-0.5 views come from the scale stage's outputs
    assert np.array_equal(np.unique(many.view_scale), [0.5, 1.0])
    del torch


def test_fast_tile_flags_are_conservative():
    """The planner's per-tile flags never skip work that matters: every corner that passes the
    content filter (oracle, on oracle views) lies in a tile marked for detection, and every
    pixel within 21 px of such a corner (the BRIEF reach) or with mask 1 lies in a tile marked
    for smoothing; on tilted views a sizable share of tiles skips detection."""
    import synth
    from oracle import orb as OO
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    img = case.A
    rows = [(1.0, 0.0), (2.0, 0.3), (2.0, 1.9), (2.0 * math.sqrt(2), 0.7), (4.0, 1.2), (4.0, 2.8)]
    L = 4
    plan = X.plan_image(img.shape[1], img.shape[0], X.make_params(rows), L, 1.2, 300, 20)
    h = plan.header
    vl = np.frombuffer(plan.blob, np.int32, plan.n_views * L + 1, int(h["off_vl_prefix"]))
    flags = np.frombuffer(plan.blob, np.uint8, int(vl[-1]), int(h["off_fast_flags"]))
    skipped = 0
    for i, (t, phi) in enumerate(rows):
        v = OP.plan_view(img.shape[1], img.shape[0], t, phi)
        _, M, U = OS.simulate_view(img, v)
        dims = OP.level_dims(v.width, v.height, L)
        for l, (P, Mk) in enumerate(OO.build_pyramid(U, M, dims)):
            W, H = dims[l]
            tx_n = (W + 63) // 64
            f = flags[vl[i * L + l]:vl[i * L + l + 1]].reshape(-1, tx_n)
            skipped += int(((f & 2) == 0).sum())
            ys, xs = np.nonzero(Mk)
            assert np.all(f[ys // 32, xs // 64] & 1), (i, l)
            cx, cy = OO.fast_candidates(P, Mk, 20)
            assert np.all(f[cy // 32, cx // 64] & 2), (i, l)
            for x, y in zip(cx, cy):
                for yy in (max(0, y - 21), min(H - 1, y + 21)):
                    for xx in (max(0, x - 21), min(W - 1, x + 21)):
                        assert f[yy // 32, xx // 64] & 1, (i, l, x, y)
    print("tiles without detection", skipped, "of", len(flags))
    assert skipped > 0.2 * len(flags)


def test_scaled_grid_matches_oracle_and_interp_switch():
    g = X.sampling_grid(5, 72.0, 0.5)
    ref = OP.sampling_grid_scaled(5, 0.5)
    assert len(g) == len(ref) == 45
    for r, (t, phi, s) in zip(g, ref):
        assert r["t"] == t and abs(r["phi"] - phi) < 1e-15 and r["s"] == s
    assert np.array_equal(X.sampling_grid(5, 72.0, 0.0), X.sampling_grid(5))
    with pytest.raises(X.XAError):
        X.sampling_grid(5, 72.0, -0.5)
    p = X.plan_image(64, 48, X.make_params([(1.0, 0.0), (2.0, 0.5)]), 2, 1.2, 50, 20, interp="nearest")
    assert np.all(p.views["interp"] == 1)
    assert np.all(X.plan_image(64, 48, X.make_params([(2.0, 0.5)]), 2, 1.2, 50, 20).views["interp"] == 0)
    with pytest.raises(X.XAError):
        X._check(X.lib().xa_plan_set_interp(p.blob.ctypes.data, 7))


def test_warp_stride_residues(L):
    """The planner's LDS row-stride residue of each view: in 0..63, the same for views that share
    a linear map and tile width (one search per map), and deterministic."""
    g = X.sampling_grid(5)
    p1 = X.plan_image(1024, 768, g, 8, 1.2, 1000, 20)
    p2 = X.plan_image(1024, 768, g, 8, 1.2, 1000, 20)
    p3 = X.plan_image(900, 700, g, 8, 1.2, 1000, 20)
    m1 = p1.views["warp_ls_mod"]
    assert ((m1 >= 0) & (m1 < 64)).all()
    assert np.array_equal(m1, p2.views["warp_ls_mod"])
    # blurred views carry the blur's outputs per thread (the default 8), unblurred ones 0
    assert (p1.views["blur_rows"] == np.where(p1.views["sigma"] > 0, 8, 0)).all()
    # a second image size gives the same linear maps: each residue lies in 0..63 there too
    assert ((p3.views["warp_ls_mod"] >= 0) & (p3.views["warp_ls_mod"] < 64)).all()
    # duplicated grid views share the residue
    rows = [(2.0, 0.5), (2.0, 0.5), (1.0, 0.0)]
    p4 = X.plan_image(300, 200, X.make_params(rows), 3, 1.2, 100, 20)
    assert p4.views["warp_ls_mod"][0] == p4.views["warp_ls_mod"][1]


def test_check_reports_runtime_state(L):
    """xa_check returns a status and a message and never crashes: XA_OK on a healthy runtime, and
    XA_EHIP naming the runtime's error where no GPU is present (as in this CPU-only container)."""
    import torch
    st = L.xa_check(None)
    msg = L.xa_last_error().decode()
    if torch.cuda.is_available():
        assert st == X.XA_OK and msg == ""
    else:
        assert st == X.XA_EHIP and "device" in msg
    # a host-rejected argument error leaves nothing pending for xa_check
    assert L.xa_match_views(256, 256, 0, 256, 256, 1, 100, 4, 5, 256, 256, 256, None) == X.XA_EINVAL
    assert L.xa_check(None) == st


def test_warp_tile_table_drives_the_planner(L):
    """xa_set_warp_tiles: widths per compression class, validated, used by plans made afterwards
    only; NULL restores the built-in rule (16 below t/s = 2, 8 below 8, else 4)."""
    rule = X.get_warp_tiles()
    assert rule.tolist() == [16, 16, 8, 8, 8, 8, 4, 4]
    grid = X.sampling_grid(5)
    before = X.plan_image(640, 480, grid, 3, 1.2, 300, 20)
    try:
        X.set_warp_tiles([32, 16, 8, 8, 4, 4, 64, 4])
        assert X.get_warp_tiles().tolist() == [32, 16, 8, 8, 4, 4, 64, 4]
        p = X.plan_image(640, 480, grid, 3, 1.2, 300, 20)
        want = {1.0: 32, 1.414: 16, 2.0: 8, 2.828: 8, 4.0: 4, 5.657: 4}
        for v in p.views:
            assert v["warp_tile_w"] == want[round(float(v["p"]["t"]), 3)]
        # the class is that of the compression t / s: t = 8 is class 6, t = 4 magnified by s = 2 class 2
        p2 = X.plan_image(640, 480, X.make_params([(8.0, 0.0, 0.0, 1.0), (4.0, 0.0, 0.0, 2.0)]), 3, 1.2, 300, 20)
        assert p2.views["warp_tile_w"].tolist() == [64, 8]
        # tiles of a view cover it: the warp prefix counts ceil(W / w) ceil(H / (512 / w)) per view
        wp = np.frombuffer(p.blob, np.int32, p.n_views + 1, int(p.header["off_warp_prefix"]))
        for i, v in enumerate(p.views):
            w = int(v["warp_tile_w"])
            assert wp[i + 1] - wp[i] == -(-int(v["width"]) // w) * -(-int(v["height"]) // (512 // w))
        for bad in ([3] + [0] * 7, [0] * 7 + [128]):
            with pytest.raises(X.XAError):
                X.set_warp_tiles(bad)
        # plans made before keep their widths
        assert before.views["warp_tile_w"][0] == 16
    finally:
        X.set_warp_tiles(None)
    assert X.get_warp_tiles().tolist() == rule.tolist()
    assert X.lib().xa_tune_warp_tiles_workspace_size(8, 8) == 0
    assert X.lib().xa_tune_warp_tiles_workspace_size(1024, 768) > 1024 * 768


def test_blur_rows_table_drives_the_planner(L):
    """xa_set_blur_rows: the blur's outputs per thread (4 or 8) per compression class, validated,
    used by plans made afterwards only, with blur tiles of 64 x 4r (taps along x) or 4r x 64 counted
    in the plan's blur prefix; NULL restores 8 everywhere."""
    assert X.get_blur_rows().tolist() == [8] * 8
    grid = X.sampling_grid(5)
    before = X.plan_image(640, 480, grid, 3, 1.2, 300, 20)
    try:
        X.set_blur_rows([0, 4, 8, 4, 8, 4, 8, 8])
        assert X.get_blur_rows().tolist() == [8, 4, 8, 4, 8, 4, 8, 8]
        p = X.plan_image(640, 480, grid, 3, 1.2, 300, 20)
        want = {1.414: 4, 2.0: 8, 2.828: 4, 4.0: 8, 5.657: 4}
        v = p.views
        blurred = np.nonzero(v["sigma"] > 0)[0]
        for i in blurred:
            assert v["blur_rows"][i] == want[round(float(v["p"]["t"][i]), 3)]
        assert (v["blur_rows"][v["sigma"] == 0] == 0).all()
        bp = np.frombuffer(p.blob, np.int32, len(blurred) + 1, int(p.header["off_blur_prefix"]))
        for j, i in enumerate(blurred):
            r = int(v["blur_rows"][i])
            tw, th = (64, 4 * r) if v["blur_major"][i] == 0 else (4 * r, 64)
            assert bp[j + 1] - bp[j] == -(-int(v["src_w"][i]) // tw) * -(-int(v["src_h"][i]) // th)
        for bad in ([2] + [0] * 7, [0] * 7 + [16]):
            with pytest.raises(X.XAError):
                X.set_blur_rows(bad)
        assert (before.views["blur_rows"][before.views["sigma"] > 0] == 8).all()
    finally:
        X.set_blur_rows(None)
    assert X.get_blur_rows().tolist() == [8] * 8
    assert X.lib().xa_tune_blur_rows_workspace_size(8, 8) == 0
    assert X.lib().xa_tune_blur_rows_workspace_size(1024, 768) > 1024 * 768
