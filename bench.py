"""Benchmark: image pairs per second through the whole parameter-search path on one MI355X.

A step is one call of the batched entry point (xa_match_batch) on the full-size
synthetic pair: both 1024x768 / 725x725 images are simulated over the 45-view
grid (tilts sqrt(2)^0..5, longitude step 72/t) as one view plan, ORB (8 levels
at 1.2, 1000 keypoints per view, FAST threshold 20) runs on all 90 views, all
45 x 45 view pairs are matched with a 0.8 ratio test and the best pair is
selected.  Inputs are resident in device memory before timing starts.

Prints one JSON line.  Besides the headline it reports, for the all-pairs
Hamming matcher (the variant the autotuner picks: the fp4 matrix-core kernel,
priced as a +-1 contraction of 256 multiply-adds per descriptor comparison
against the dense fp4 MFMA peak, or a popcount kernel, priced in integer
lane-ops against the vector-ALU peak), its achieved rate timed with HIP events
on the launch stream, and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 64 lane-ops / clock / CU
VALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK_BPS = 8.0e12
HAMMING_OPS_PER_CMP = 16          # 8 x v_xor_b32 + 8 x v_bcnt_u32_b32 per 256-bit comparison
# dense fp4 MFMA peak of the MI355X (no sparsity): 10.1 PFLOP/s
FP4_PEAK_FLOPS = 10.1e15
MX_FLOPS_PER_CMP = 2 * 256        # a +-1 dot product of two 256-bit descriptors: 256 multiply-adds
MATCH_MATRIX = -1                 # matcher variant code of the matrix-core kernel
MATCH_MATRIX_PACKED = -2          # the same with query tiles packed across views

# HBM traffic of the matching kernel on the full-size pair, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) per matcher variant (-1 = the matrix-core
# kernel, else the popcount kernel's queries per lane), scaled by what the same
# counters read for a plain 1 GiB device-to-device copy (FETCH_SIZE reads 0.5 GiB there,
# WRITE_SIZE 1 GiB).  Valid only for the matcher source it was measured on: any change to that
# file reports null.
K_MATCH_TRAFFIC = {
    "source": "paper_2503_03479_amd/csrc/match.hip",
    "sha256": "8b70214ddfeb76df949cb1d274d3e94e0e95729e6216c522fc9172ede0600971",
    "fetch_scale": 2.0, "write_scale": 1.0,
    # variant -> (fetch, write), all measured on this source
    "kib": {-1: (8162.3, 15619.2), -2: (10932.1, 17123.9), 1: (6714.1, 15745.8), 2: (8086.2, 15619.2),
            4: (10855.9, 15555.9)},
}


def k_match_traffic(queries_per_lane: int):
    import hashlib
    t = K_MATCH_TRAFFIC
    if queries_per_lane not in t["kib"]:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    fetch, write = t["kib"][queries_per_lane]
    return (fetch * t["fetch_scale"] + write * t["write_scale"]) * 1024.0


# HBM traffic of k_warp on one launch over both images' 90 views of the full-size pair (the launch
# the timed step makes), from the same two --pmc passes and copy calibration as the matcher's, with
# the warp tile widths given here (the tuner's usual choice on MI355X).  Valid only for the simulate
# sources it was measured on and for those widths.
K_WARP_TRAFFIC = {
    "sources": ["paper_2503_03479_amd/csrc/simulate.hip", "paper_2503_03479_amd/csrc/internal.h",
                "paper_2503_03479_amd/csrc/lanczos.h"],
    "sha256": "890a880b91694d9cd60d69d982a8926e567cfe6571c386653cdb33d4eec97525",   # of the sources, concatenated
    "warp_tiles": [32, 16, 8, 8, 8, 8, 8, 8],
    "fetch_scale": 2.0, "write_scale": 1.0,
    "kib": (109313.8, 67581.6),   # (fetch, write) per launch
}
WARP_OPS_PER_PX = 72 + 16         # 64 + 8 multiply-adds of the 8 x 8 sum and the 16 kernel weights per view pixel


def k_warp_traffic():
    import hashlib
    from paper_2503_03479_amd import xaffine as X
    t = K_WARP_TRAFFIC
    if [int(w) for w in X.get_warp_tiles()] != t["warp_tiles"]:
        return None
    h = hashlib.sha256()
    for src in t["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t["sha256"]:
        return None
    fetch, write = t["kib"]
    return (fetch * t["fetch_scale"] + write * t["write_scale"]) * 1024.0


def warp_roofline(case, grid_np, wl, dev, stream, pattern, match_stage, reps: int = 20, warmup: int = 5):
    """The dominant kernel, k_warp, on exactly the launch of the timed step: one xa_warp_views call over
    both images' views (one view plan over one sources buffer), its blurred planes made once by
    xa_blur_views, timed with HIP events on the launch stream around each warp launch inside a
    step-like sequence of launches.  Algorithmic work per view pixel:
    the 8 x 8 weighted sum and its 8 row sums (72 multiply-adds) and the 16 kernel weights; algorithmic
    bytes: each source read once per view (fp32 when blurred, else u8) and the canvas and mask written."""
    import numpy as np
    import torch
    from paper_2503_03479_amd import xaffine as X
    arena_src = X.SourceArena()
    ia = arena_src.add(case.A.shape[1], case.A.shape[0])
    ib = arena_src.add(case.B.shape[1], case.B.shape[0])
    buf = torch.from_numpy(arena_src.pack({ia: case.A, ib: np.ascontiguousarray(case.B)})).to(dev)
    params = np.concatenate([grid_np, grid_np])
    plan = X.plan_views(arena_src.table(), [ia] * len(grid_np) + [ib] * len(grid_np), params, wl["n_levels"], 1.2,
                        wl["n_features"], wl["fast"])
    arena = torch.zeros(plan.arena_bytes, dtype=torch.uint8, device=dev)
    mask = torch.zeros(plan.arena_bytes, dtype=torch.uint8, device=dev)
    ws = X._empty(X.lib().xa_simulate_workspace_size(plan.host_ptr()), dev)
    X.blur_views(plan, buf, ws)
    X.warp_views(plan, buf, arena, mask, ws)
    torch.cuda.synchronize()
    ext_ws = X._empty(X.lib().xa_extract_workspace_size(plan.host_ptr()), dev)
    # each timed warp launch sits in a whole step's sequence of launches (blur, warp, ORB, matching),
    # as in the timed region: warps launched back to back alone run hotter and slower.  Only the
    # warp launches sit between the events.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps + warmup)]
    for e0, e1 in ev:
        X.blur_views(plan, buf, ws)
        e0.record(stream)
        X.warp_views(plan, buf, arena, mask, ws)
        e1.record(stream)
        X.extract_orb(plan, arena, mask, pattern, ws=ext_ws)
        match_stage()
    torch.cuda.synchronize()
    t = sum(e0.elapsed_time(e1) for e0, e1 in ev[warmup:]) / reps / 1e3      # the first `warmup` untimed
    v = plan.views
    px = int((v["width"].astype(np.int64) * v["height"]).sum())
    src_px = np.array([int(d["width"]) * int(d["height"]) for d in arena_src.table()])[v["source"]]
    algo_bytes = int(np.where(v["sigma"] > 0, 4 * src_px, src_px).sum()) + 2 * px
    ops = WARP_OPS_PER_PX * px
    return {"kernel": "k_warp (xa_warp_views over both images' 90 views, one launch as in the timed step)",
            "bound": "alu", "achieved": ops / t / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
            "frac": ops / t / VALU_PEAK_OPS, "traffic": k_warp_traffic(),
            "traffic_unit": "bytes per launch (HBM, counter-measured)",
            "algorithmic_ops_per_launch": ops, "algorithmic_bytes_per_launch": algo_bytes,
            "view_px_per_launch": px, "ms_per_launch": t * 1e3,
            "hbm_GBps": algo_bytes / t / 1e9, "hbm_frac": algo_bytes / t / HBM_PEAK_BPS}


def progress(msg: str):
    print(msg, file=sys.stderr, flush=True)


def profiler_preloaded() -> bool:
    """True when a profiler's tool library is preloaded into this process (rocprofv3 and its kin
    set LD_PRELOAD and ROCPROF_* / ROCP_* variables).  Such a tool initialises the GPU before the
    program starts, so this process must not start worker processes: each would be a fork and exec
    of a process that has already touched the GPU."""
    if "rocprof" in os.environ.get("LD_PRELOAD", ""):
        return True
    return any(k.startswith(("ROCPROF_", "ROCP_")) for k in os.environ)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["full", "tiny"], default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-pairs", type=int, default=64, help="image pairs in the batched leg (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes rendering the batched leg's pairs (0 = in this process, one progress "
                         "line per pair; for profiler runs, which would otherwise load the profiler into "
                         "every worker)")
    ap.add_argument("--crops", type=int, default=256, help="crops in the differentiable-warp leg (0 = skip)")
    ap.add_argument("--matcher-q", type=int, default=0, choices=[0, 1, 2, 4, MATCH_MATRIX, MATCH_MATRIX_PACKED],
                    help="matcher variant for the full-pair leg: 0 = autotune, 1 / 2 / 4 = popcount kernel "
                         "with that many queries per lane, -1 = matrix-core kernel")
    ap.add_argument("--l2-n", type=int, default=32768, help="descriptors per set in the L2 matcher leg (0 = skip)")
    ap.add_argument("--no-sift", action="store_true", help="skip the SIFT leg")
    ap.add_argument("--no-sweep", action="store_true", help="skip the Sec. IV.D sweep leg")
    ap.add_argument("--no-tune-tiles", action="store_true",
                    help="keep the built-in warp tile widths and blur outputs per thread")
    ap.add_argument("--blur-rows", default=None,
                    help="fixed blur outputs per thread per compression class, 8 comma-separated values from 4 8 "
                         "(instead of tuning them)")
    ap.add_argument("--warp-tiles", default=None,
                    help="fixed warp tile widths per compression class, 8 comma-separated values from 4 8 16 32 "
                         "64 (instead of tuning them; for runs under a profiler, which distorts the tuner's timings)")
    ap.add_argument("--only", choices=["batched", "diffwarp", "copy", "sweep", "l2", "sift"], default=None,
                    help="run one leg alone and print its JSON (for profiler runs); 'copy' is a plain 1 GiB "
                         "device-to-device copy whose counter readings calibrate the HBM traffic counters")
    return ap.parse_args()


WORKLOADS = {
    "full": dict(n_tilt=5, n_levels=8, n_features=1000, fast=20),
    "tiny": dict(n_tilt=2, n_levels=3, n_features=300, fast=20),
}


# ---------------------------------------------------------------- oracle on all host cores
# The whole oracle pipeline of one pair, split into independent tasks (simulate + ORB per view,
# then one row of the view-pair matching table per task) over a pool of worker processes with
# one BLAS / OpenMP thread each.  The pool is started before this process touches the GPU.

_CPU_CTX = {}


def _cpu_workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_init(ctx):
    _CPU_CTX.clear()
    _CPU_CTX.update(ctx)


def _cpu_view_task(task):
    """(key, i) -> (key, i, descriptors, seconds): oracle simulate + ORB of view i of image key."""
    from oracle import orb as OO
    from oracle import plan as OP
    from oracle import simulate as OS
    key, i = task
    c = _CPU_CTX
    t0 = time.perf_counter()
    img = c[key]
    t, f = c["grid"][i]
    v = OP.plan_view(img.shape[1], img.shape[0], t, f)
    V, mask, U = OS.simulate_view(img, v)
    dims = OP.level_dims(v.width, v.height, c["n_levels"])
    fe = OO.extract_view(U, mask, dims, c["quotas"], c["fast"], c["pattern"])
    return key, i, fe["desc"], time.perf_counter() - t0


def _cpu_match_task(task):
    """(i, desc_a_i, descs_b) -> (i, counts over j, seconds): oracle matching of view i of A
    against every view of B with the ratio test 4/5."""
    from oracle import match as OM
    i, da, dbs = task
    t0 = time.perf_counter()
    counts = []
    for db in dbs:
        idx, d1, d2 = OM.nearest_two(da, db)
        counts.append(int(OM.ratio_accept(d1, d2, len(db), 4, 5).sum()))
    return i, counts, time.perf_counter() - t0


def _cpu_crop_task(task):
    """(crop, params, gout) -> seconds: the oracle's fp64 forward and adjoint of one crop."""
    from oracle import diffwarp as OD
    crop, P, g = task
    t0 = time.perf_counter()
    OD.warp_forward(crop, P)
    OD.warp_adjoint(crop, g, P)
    return time.perf_counter() - t0


def _cpu_context(name):
    import numpy as np

    import synth
    from oracle import plan as OP
    wl = WORKLOADS[name]
    case = synth.make_pair(**synth.PAIR_CONFIGS[name])
    grid = [(float(t), float(f)) for t, f in OP.sampling_grid(wl["n_tilt"])]
    return {"a": case.A, "b": np.ascontiguousarray(case.B), "grid": grid, "n_levels": wl["n_levels"],
            "quotas": OP.level_quotas(wl["n_features"], wl["n_levels"]), "fast": wl["fast"],
            "pattern": synth.brief_pattern()}


def _cpu_pair(pool, ctx, pick=None):
    """The oracle's parameter search for one pair on the pool, whose workers hold ctx, over the
    views `pick` of each image (all by default) and every view pair among them: (wall seconds,
    seconds per view, seconds per view pair (summed over the workers' tasks), best pair)."""
    n = len(ctx["grid"])
    pick = list(range(n)) if pick is None else list(pick)
    t0 = time.perf_counter()
    views = pool.map(_cpu_view_task, [(k, i) for k in ("a", "b") for i in pick], chunksize=1)
    feats = {"a": {}, "b": {}}
    t_view = 0.0
    for key, i, d, dt in views:
        feats[key][i] = d
        t_view += dt
    rows = pool.map(_cpu_match_task, [(i, feats["a"][i], [feats["b"][j] for j in pick]) for i in pick],
                    chunksize=1)
    wall = time.perf_counter() - t0
    best, t_match = (-1, -1, -1), 0.0
    for i, counts, dt in sorted(rows):
        t_match += dt
        for jj, c in enumerate(counts):
            if c > best[2]:
                best = (i, pick[jj], c)
    return wall, t_view / (2 * len(pick)), t_match / (len(pick) ** 2), best


def cpu_baselines():
    """The oracle timed on the host's cores (a spawn pool, one thread per worker).  Headline: the
    full-size pair's search on a sample of 12 evenly spaced views of each image and the 144 view
    pairs among them, scaled to the whole search (90 views, 2025 view pairs) by its measured
    seconds per view and per view pair, at the sample's own parallel efficiency.  Also: the tiny
    pair's whole search (median of 3) and 4 of the 256 differentiable-warp crops (fp64 forward +
    adjoint)."""
    import multiprocessing as mp

    import numpy as np

    import synth
    workers = _cpu_workers()
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        sp = mp.get_context("spawn")
        progress(f"cpu baseline: oracle on {workers} worker processes")
        ctx = _cpu_context("full")
        nv = len(ctx["grid"])
        pick = sorted(set(int(round(x)) for x in np.linspace(0, nv - 1, 12)))
        with sp.Pool(workers, initializer=_cpu_init, initargs=(ctx,)) as pool:
            wall_s, t_view, t_match, best = _cpu_pair(pool, ctx, pick)
        work_s = t_view * 2 * len(pick) + t_match * len(pick) ** 2
        work_full = t_view * 2 * nv + t_match * nv * nv
        wall_full = wall_s * work_full / work_s
        progress(f"cpu baseline: full-pair sample {wall_s:.1f} s wall, {work_s:.1f} s of work")
        ctx = _cpu_context("tiny")
        tiny = []
        with sp.Pool(workers, initializer=_cpu_init, initargs=(ctx,)) as pool:
            for _ in range(3):
                w_, tv, tm, _ = _cpu_pair(pool, ctx)
                m = len(ctx["grid"])
                tiny.append((w_, tv * 2 * m + tm * m * m))
        tiny = sorted(tiny)[1]
        with sp.Pool(min(4, workers)) as pool:
            crops = synth.make_crops(4, 512, 5000, distinct=4)
            P = synth.crop_params(256, 5000)[:4]
            g = synth.rng(5).standard_normal(crops.shape).astype(np.float32)
            t0 = time.perf_counter()
            per_crop = pool.map(_cpu_crop_task, [(crops[k], P[k], g[k]) for k in range(4)], chunksize=1)
            dw_wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {
        "value": 1.0 / wall_full, "unit": "pairs/s", "cores": workers, "kind": "oracle",
        "sample": f"the full-size pair: simulate + ORB of {len(pick)} evenly spaced views of each image "
                  f"({t_view:.2f} s per view) and the {len(pick) ** 2} view-pair matchings among them "
                  f"({t_match * 1e3:.1f} ms each) on {workers} worker processes with one thread each, "
                  f"{wall_s:.1f} s wall for {work_s:.1f} s of work; scaled to {2 * nv} views and {nv * nv} view pairs",
        "seconds_per_pair": wall_full, "single_core_seconds_per_pair": work_full,
        "single_core_value": 1.0 / work_full, "sample_best_pair": list(best),
        "configs": {
            "tiny": {"pairs_per_s": 1.0 / tiny[0], "single_core_pairs_per_s": 1.0 / tiny[1], "cores": workers,
                     "sample": "the tiny pair's whole search, median of 3"},
            "diffwarp": {"crops_per_s": 4 / dw_wall, "single_core_crops_per_s": 4 / sum(per_crop), "cores": min(4, workers),
                         "sample": "fp64 forward + adjoint of 4 of the 256 crops of 512x512, one per worker"},
        },
        "host_cpu": platform.processor() or platform.machine(), "host_cpu_count": os.cpu_count(),
    }


def _make_batch_pair(k):
    import synth
    p = synth.batch_pairs(1, seed=3000 + k)[0]
    return p.A, p.B, p.meta


def batched_leg(args, dev, pattern, raw, gen_s):
    """Many pairs of uneven sizes (sides 480..2048, aspect 0.6..1.6, absolute tilt 0..80 deg),
    45-view grid at scales 1 and 1/2, 8 levels, 500 keypoints: all pairs in one graph replay
    (views in memory-bounded chunks, one matching launch) against the same pairs run one
    after another through the same entry point, one synchronisation per pair."""
    import numpy as np
    import torch

    from paper_2503_03479_amd import xaffine as X

    K = len(raw)
    pairs = [(A, np.ascontiguousarray(B)) for A, B, _ in raw]
    grid = [(float(r["t"]), float(r["phi"])) for r in X.sampling_grid(5)]
    kw = dict(n_levels=8, n_features=500, fast_threshold=20, device=dev, queries_per_lane="auto")
    stream = torch.cuda.current_stream()

    # the batch first: its first run tunes the matcher on its own descriptors
    batch = X.BatchRunner(pairs, grid, (1.0, 0.5), **kw)
    batch.run(pattern)
    torch.cuda.synchronize()
    progress("batched leg: first batch run (matcher tuned) done")
    steps = max(1, args.batch_steps)

    # plain: one runner per pair (same entry point and matcher variant, one pair per call), one
    # shared workspace
    kw1 = dict(kw, queries_per_lane=batch.mplan_q)
    single = [X.BatchRunner([pr], grid, (1.0, 0.5), allocate_ws=False, **kw1) for pr in pairs]
    shared = X._empty(max(r.ws_bytes for r in single), dev)
    for r in single:
        r.set_workspace(shared)
    for r in single[:2]:
        r.run(pattern)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in single:
            r.run(pattern)
            torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / steps
    del shared
    progress("batched leg: per-pair runs timed")

    # the plain path fixed up front for this comparison: the same kernels, one launch per stage
    # per view (the scale stage once per pair, simulate and ORB on one-view plans, matching one
    # view of A against all of B's views per call), one host synchronisation per pair, no graph
    pv = _plain_per_view_setup(X, batch, dev)
    _plain_per_view_run(X, batch, pv, pattern, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for k in range(K):
            _plain_per_view_run(X, batch, pv, pattern, k)
            torch.cuda.synchronize()
    per_view_s = (time.perf_counter() - t0) / steps
    progress("batched leg: per-view plain path timed")

    batch.capture(pattern)
    batch.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        batch.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / steps
    batch_ev_s = e0.elapsed_time(e1) / 1e3 / steps
    batch.close()
    progress("batched leg: graph replays timed")

    # the batch reproduces the per-pair results exactly
    same = True
    for k, r in enumerate(single):
        a0, na, b0, nb = batch.pair_views[k]
        base = int(batch.mplan.groups[k]["pair_base"])
        same &= bool(torch.equal(batch.best[k], r.best[0]))
        same &= bool(torch.equal(batch.pair_count[base:base + na * nb], r.pair_count))
        same &= bool(torch.equal(batch.desc[a0:a0 + na], r.desc[:na]))
    same_pv = bool(torch.equal(batch.pair_count, pv["pair_count"])) and bool(torch.equal(batch.desc, pv["desc"])) \
        and bool(torch.equal(batch.count, pv["count"]))
    sides = [(A.shape[1], A.shape[0], B.shape[1], B.shape[0]) for A, B in pairs]
    comparisons = 0
    counts = batch.count.cpu().numpy().astype(np.int64)
    for (a0, na, b0, nb) in batch.pair_views:
        comparisons += int(counts[a0:a0 + na].sum() * counts[b0:b0 + nb].sum())
    return {
        "workload": f"{K} pairs, sides 480..2048 (aspect 0.6..1.6), absolute tilt 0..80 deg, 45-view grid at "
                    f"scales 1 and 1/2 (90 views per image), 8 levels, 500 keypoints, ratio 4/5",
        "pairs_per_s_batched": K / batch_s,
        "pairs_per_s_plain": K / plain_s,
        "batched_over_plain": plain_s / batch_s,
        "pairs_per_s_plain_per_view": K / per_view_s,
        "batched_over_plain_per_view": per_view_s / batch_s,
        "plain_per_view": "the same kernels, one launch per stage per view: the scale stage once per pair, simulate "
                          "and ORB on a one-view plan for each of the pair's 180 views, matching one view of A "
                          "against B's 90 views per call; a host synchronisation after each pair, no graph",
        "plain_per_view_launch_calls_per_pair": pv["calls_per_pair"],
        "identical_to_plain_per_view": same_pv,
        "ms_per_batch": batch_s * 1e3,
        "event_ms_per_batch": batch_ev_s * 1e3,
        "ms_per_pair_plain": plain_s * 1e3 / K,
        "plain": "the same entry point with one pair per call and a host synchronisation after each pair",
        "batched": "one HIP graph replay: scale stage, then simulate + ORB in memory-bounded view chunks, then "
                   "one matching launch over all pairs' view pairs",
        "views": batch.n_views,
        "chunks": len(batch.chunks),
        "workspace_GiB": batch.ws.numel() / 2 ** 30,
        "comparisons": comparisons,
        "identical_to_plain": same,
        "matcher_autotune": batch.autotune,
        "mean_side_px": float(np.mean([math.sqrt(a * b) for a, b, _, _ in sides])),
        "generate_s": gen_s,
    }


def _plain_per_view_setup(X, batch, dev):
    """One-view plans for every view of the batch (in its numbering), per-pair scale plans, and
    buffers of the batch's shapes for the plain per-view path."""
    import numpy as np
    import torch
    L = X.lib()
    table = batch.arena.table()
    N = batch.mplan.n_features
    plans = []
    for v in range(batch.n_views):
        p = X.plan_views(table, [batch.view_source[v]], np.array([batch.view_rows[v % len(batch.view_rows)]],
                                                                   X.PARAMS_DTYPE), 8, 1.2, N, 20)
        plans.append((p, X._ptr(p.device(dev))))
    splans = []
    for jobs in batch.pair_jobs:
        sp = X.plan_scales(np.array(jobs, X.SCALE_JOB_DTYPE)) if jobs else None
        splans.append((sp, X._ptr(sp.device(dev)) if sp else None))
    arena_bytes = max(p.arena_bytes for p, _ in plans)
    ws_bytes = max(max(L.xa_simulate_workspace_size(p.host_ptr()), L.xa_extract_workspace_size(p.host_ptr()))
                   for p, _ in plans)
    ws_bytes = max([ws_bytes] + [L.xa_scale_workspace_size(sp.host_ptr()) for sp, _ in splans if sp])
    nv = batch.n_views
    z = lambda *sh, dt=torch.uint8: torch.zeros(sh, dtype=dt, device=dev)  # noqa: E731
    pv = {"plans": plans, "splans": splans, "arena": z(arena_bytes), "mask": z(arena_bytes), "ws": X._empty(ws_bytes, dev),
          "sources": batch.sources.clone(), "kp": z(nv, N, 40), "desc": z(nv, N, 32), "count": z(nv, dt=torch.int32),
          "matches": z(batch.mplan.total_pairs, N, 8), "pair_count": z(batch.mplan.total_pairs, dt=torch.int32),
          "best": z(4, dt=torch.int32), "N": N}
    a0, na, b0, nb = batch.pair_views[0]
    pv["calls_per_pair"] = {"scale": 1 if splans[0][0] else 0, "simulate": na + nb, "extract": na + nb, "match": na}
    return pv


def _plain_per_view_run(X, batch, pv, pattern, k):
    """Pair k through the plain per-view path (asynchronous; the caller synchronises)."""
    L = X.lib()
    st = X._stream()
    N = pv["N"]
    ws, wsb = X._ptr(pv["ws"]), pv["ws"].numel()
    src = X._ptr(pv["sources"])
    sp, spd = pv["splans"][k]
    if sp:
        X._check(L.xa_scale_sources(sp.host_ptr(), spd, src, None, ws, wsb, st))
    a0, na, b0, nb = batch.pair_views[k]
    arena, mask, pat = X._ptr(pv["arena"]), X._ptr(pv["mask"]), X._ptr(pattern)
    kp, desc, count = pv["kp"], pv["desc"], pv["count"]
    for v in list(range(a0, a0 + na)) + list(range(b0, b0 + nb)):
        p, pd = pv["plans"][v]
        X._check(L.xa_simulate_views(p.host_ptr(), pd, src, arena, mask, None, ws, wsb, st))
        X._check(L.xa_extract_orb(p.host_ptr(), pd, arena, mask, pat, X._ptr(kp[v]), X._ptr(desc[v]),
                                  X._ptr(count[v:v + 1]), ws, wsb, st))
    base = int(batch.mplan.groups[k]["pair_base"])
    for i in range(na):
        q = base + i * nb
        X._check(L.xa_match_views(X._ptr(desc[a0 + i]), X._ptr(count[a0 + i:a0 + i + 1]), 1, X._ptr(desc[b0]),
                                  X._ptr(count[b0:b0 + nb]), nb, N, 4, 5, X._ptr(pv["matches"][q]),
                                  X._ptr(pv["pair_count"][q:q + nb]), X._ptr(pv["best"]), st))


def sweep_leg(args, dev, pattern):
    """The parameter studies of Sec. IV.D as timings on the full-size pair, in the paper's search
    mode (nearest-neighbour views of A over the grid with s_i = 1 + i ds, matched against B's
    identity view): ORB point count N in {500, 800, 1000, 1200, 1500} at ds = 0.5, and
    ds in {0, 0.2, ..., 1.0} at N = 1000.  Per setting: ms per pair (HIP events, 10 calls),
    views and their pixels, best-pair matches and precision at 2 px."""
    import numpy as np
    import torch

    import synth
    from paper_2503_03479_amd import xaffine as X

    case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
    A = torch.from_numpy(np.ascontiguousarray(case.A)).to(dev)
    Bn = np.ascontiguousarray(case.B)
    B = torch.from_numpy(Bn).to(dev)
    stream = torch.cuda.current_stream()
    out = []
    settings = [(n, 0.5) for n in (500, 800, 1000, 1200, 1500)] + [(1000, ds) for ds in (0.0, 0.2, 0.4, 0.6, 0.8, 1.0)]
    for n, ds in settings:
        grid = X.sampling_grid(5, 72.0, ds)
        pa = X.plan_image(1024, 768, grid, 8, 1.2, n, 20, interp="nearest")
        pb = X.plan_image(Bn.shape[1], Bn.shape[0], X.make_params([(1.0, 0.0)]), 8, 1.2, n, 20, interp="nearest")
        run = X.PairRunner(pa, pb, dev)
        run.run(A, B, pattern)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            run.run(A, B, pattern)
        e1.record(stream)
        torch.cuda.synchronize()
        pr = run.precision(case.H, 2.0).cpu().numpy()
        out.append({"n_features": n, "delta_s": ds, "ms_per_pair": e0.elapsed_time(e1) / 10,
                    "views": pa.n_views, "view_mpx": float((pa.views["width"] * pa.views["height"]).sum()) / 1e6,
                    "best_pair": run.best.cpu().numpy().tolist(), "correct": int(pr[0]), "matches": int(pr[1])})
        del run
    return {"workload": "full-size pair, search mode: nearest-neighbour views of A over the 45-view grid with "
                        "s_i = 1 + i ds, single-image matching against B, 8 levels", "settings": out}


INT8_PEAK_OPS = 5.0e15            # MI355X dense int8 matrix-core peak, ops/s
L2_OPS_PER_CMP = 2 * 128          # multiply-adds of one 128-D dot product


def l2_leg(args, dev):
    """L2 nearest-two matching of 8-bit SIFT descriptors (xa_match_l2) on seeded SIFT-like sets:
    the throughput size (n x n) and the paper's size (1000 features per image), HIP events over
    10 calls after one untimed call."""
    import torch

    import synth
    from paper_2503_03479_amd import xaffine as X

    L = X.lib()
    res = {}
    for tag, n in (("large", args.l2_n), ("paper", 1000)):
        Q, T, _ = synth.sift_like_sets(n, n, 21)
        q = torch.from_numpy(Q).to(dev)
        t = torch.from_numpy(T).to(dev)
        out = torch.empty((n, 3), dtype=torch.int32, device=dev)
        count = torch.empty(1, dtype=torch.int32, device=dev)
        ws = X._empty(L.xa_match_l2_workspace_size(n, n), dev)
        stream = torch.cuda.current_stream()

        def call():
            X._check(L.xa_match_l2(X._ptr(q), n, X._ptr(t), n, 3, 4, X._ptr(out), X._ptr(count), X._ptr(ws),
                                   ws.numel(), X._stream()))

        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        cmp = n * n
        res[tag] = {"n_query": n, "n_train": n, "ms_per_call": ms, "comparisons_per_s": cmp / (ms / 1e3),
                    "accepted": int(count.cpu()[0])}
    big = res["large"]
    achieved = big["comparisons_per_s"] * L2_OPS_PER_CMP
    return {
        "workload": f"SIFT-like 8-bit descriptors (gamma magnitudes, unit length, clipped at 0.2, x512), "
                    f"half of the queries noisy copies of train rows; {args.l2_n} x {args.l2_n} and 1000 x 1000, "
                    f"ratio 3/4",
        "kernel": "k_match_l2 + k_match_l2_final (xa_match_l2, int8 matrix-core contraction)",
        "bound": "mfma", "achieved": achieved / 1e12, "peak": INT8_PEAK_OPS / 1e12, "unit": "TOP/s",
        "frac": achieved / INT8_PEAK_OPS, "ops_per_comparison": L2_OPS_PER_CMP,
        "large": big, "paper_size": res["paper"],
    }


def sift_leg(args, dev):
    """SIFT extraction (xa_extract_sift) on the full-size pair's two images, HIP events over 10
    calls after one untimed call; then the base-image selection of Sec. III.A end to end (SIFT on
    both, L2 matching both ways, eq. (1)), wall-clock with its host synchronisations; and the
    oracle's SIFT on image A, one core, for context."""
    import numpy as np
    import torch

    import synth
    from oracle import sift as OS
    from paper_2503_03479_amd import xaffine as X

    L = X.lib()
    case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
    res = {}
    stream = torch.cuda.current_stream()
    for tag, img in (("A", case.A), ("B", np.ascontiguousarray(case.B))):
        t = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
        opts = X.sift_opts()
        h, w = img.shape
        ws = X._empty(L.xa_sift_workspace_size(w, h, ctypes.byref(opts)), dev)
        kp = torch.empty((opts.max_keypoints, 8), dtype=torch.int32, device=dev)
        desc = torch.empty((opts.max_keypoints, 128), dtype=torch.uint8, device=dev)
        count = torch.empty(2, dtype=torch.int32, device=dev)

        def call():
            X._check(L.xa_extract_sift(X._ptr(t), w, h, w, ctypes.byref(opts), X._ptr(kp), X._ptr(desc), X._ptr(count),
                                       X._ptr(ws), ws.numel(), X._stream()))

        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[tag] = {"width": w, "height": h, "ms_per_image": ms, "keypoints": int(count.cpu()[0]),
                    "mpx_per_s": w * h / (ms / 1e3) / 1e6}
    A = torch.from_numpy(case.A).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(case.B)).to(dev)
    X.select_base_image(A, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        base, f1, f2 = X.select_base_image(A, B)
    torch.cuda.synchronize()
    sel_ms = (time.perf_counter() - t0) / reps * 1e3
    t0 = time.perf_counter()
    kpo, _, _ = OS.extract(case.A)
    oracle_s = time.perf_counter() - t0
    return {
        "workload": "SIFT (3 layers per octave, sigma 1.6, no doubling, contrast 0.04, edge 10, 4096 keypoints at "
                    "most) on the full-size pair's images",
        "kernels": "k_sift_hblur, k_sift_vblur, k_sift_down, k_sift_dog, k_sift_rows<0/1>, k_sift_scan, "
                   "k_sift_orient, k_sift_scan_peaks, k_sift_desc (xa_extract_sift)",
        "images": res, "base_selection_ms": sel_ms, "base": base, "f1": f1, "f2": f2,
        "oracle_s_image_a": oracle_s, "oracle_keypoints_a": int(len(kpo)), "oracle_cores": 1,
    }


def diffwarp_leg(args, dev):
    """Differentiable warp on n fp32 crops of 512 x 512 (parameters drawn per crop):
    forward and adjoint (image + six parameters) timed with HIP events."""
    import torch

    import synth
    from paper_2503_03479_amd import xaffine as X

    n = args.crops
    crops = torch.from_numpy(synth.make_crops(n, 512, 5000, distinct=16)).to(dev)
    par = torch.from_numpy(synth.crop_params(n, 5000)).to(dev)
    g = torch.randn(crops.shape, generator=torch.Generator(device=dev).manual_seed(5), device=dev)
    stream = torch.cuda.current_stream()
    L = X.lib()
    out = torch.empty_like(crops)
    mask = torch.empty(crops.shape, dtype=torch.uint8, device=dev)
    gimg = torch.empty_like(crops)
    gpar = torch.empty((n, 6), dtype=torch.float64, device=dev)
    ws = X._empty(L.xa_warp_f32_bwd_workspace_size(n, 512, 512), dev)
    wsf = X._empty(L.xa_warp_f32_fwd_workspace_size(n, 512, 512), dev)

    def fwd():
        X._check(L.xa_warp_f32_fwd(X._ptr(crops), n, 512, 512, X._ptr(par), X._ptr(out), X._ptr(mask), X._ptr(wsf),
                                   wsf.numel(), X._stream()))

    def bwd():
        X._check(L.xa_warp_f32_bwd(X._ptr(crops), X._ptr(g), X._ptr(par), n, 512, 512, X._ptr(gimg), X._ptr(gpar),
                                   X._ptr(ws), ws.numel(), X._stream()))

    res = {}
    for name, f in (("fwd", fwd), ("bwd", bwd)):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            f()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    px = n * 512 * 512
    valid = int(mask.sum())
    return {
        "workload": f"{n} fp32 crops of 512x512, t in [1, 6], phi in [0, pi), psi in [-pi, pi), s in [0.5, 1], "
                    f"shifts in [-16, 16]",
        "fwd_ms": res["fwd"], "bwd_ms": res["bwd"],
        "crops_per_s_fwd": n / (res["fwd"] / 1e3),
        # algorithmic bytes: crop read once, output (fp32) + mask (u8) written
        "fwd_GBps": px * 9 / (res["fwd"] / 1e3) / 1e9,
        # crop + output gradient read, image gradient written (its zero fill included)
        "bwd_GBps": px * 16 / (res["bwd"] / 1e3) / 1e9,
        "valid_fraction": valid / px,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported "
              f"(image pairs and views are independent; see the sharding notes in the design document)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np

    # the batched leg's pairs are rendered by worker processes before this process touches the GPU,
    # unless a profiler is preloaded (then everything runs in this process)
    if profiler_preloaded() and args.gen_workers > 0:
        progress("bench.py: profiler preloaded; rendering in this process (--gen-workers 0)")
        args.gen_workers = 0
    cpu = None
    if args.only is None and not args.no_cpu_baseline:
        if profiler_preloaded():
            progress("bench.py: profiler preloaded; no worker pool, so no oracle baseline")
        else:
            cpu = cpu_baselines()
    raw, gen_s = [], 0.0
    if args.batch_pairs > 0 and args.only in (None, "batched"):
        t0 = time.perf_counter()
        if args.gen_workers > 0:
            import multiprocessing as mp
            with mp.get_context("spawn").Pool(min(args.gen_workers, os.cpu_count() or 1)) as pool:
                raw = pool.map(_make_batch_pair, range(args.batch_pairs))
        else:
            for k in range(args.batch_pairs):
                raw.append(_make_batch_pair(k))
                progress(f"batched leg: pair {k + 1}/{args.batch_pairs} rendered")
        gen_s = time.perf_counter() - t0

    import torch

    import synth
    from paper_2503_03479_amd import xaffine as X

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    # warp tile widths per compression class, timed on this device before any plan is made
    tile_widths, tile_ms = X.get_warp_tiles(), None
    if args.warp_tiles is not None:
        X.set_warp_tiles([int(w) for w in args.warp_tiles.split(",")])
        tile_widths = X.get_warp_tiles()
    elif not args.no_tune_tiles and args.only in (None, "batched", "sweep"):
        tile_widths, tile_ms = X.tune_warp_tiles(dev)
        progress(f"bench.py: warp tile widths {tile_widths.tolist()}")
    blur_rows, blur_ms = X.get_blur_rows(), None
    if args.blur_rows is not None:
        X.set_blur_rows([int(r) for r in args.blur_rows.split(",")])
        blur_rows = X.get_blur_rows()
    elif not args.no_tune_tiles and args.only in (None, "batched", "sweep"):
        blur_rows, blur_ms = X.tune_blur_rows(dev)
        progress(f"bench.py: blur rows {blur_rows.tolist()}")
    if args.only is not None:
        pattern = torch.from_numpy(synth.brief_pattern()).to(dev)
        if args.only == "batched":
            print(json.dumps(batched_leg(args, dev, pattern, raw, gen_s)), flush=True)
        elif args.only == "l2":
            print(json.dumps(l2_leg(args, dev)), flush=True)
        elif args.only == "diffwarp":
            print(json.dumps(diffwarp_leg(args, dev)), flush=True)
        elif args.only == "sift":
            print(json.dumps(sift_leg(args, dev)), flush=True)
        elif args.only == "sweep":
            print(json.dumps(sweep_leg(args, dev, pattern)), flush=True)
        else:
            a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                              "dispatches": 3}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    cfg = synth.PAIR_CONFIGS[args.workload]
    case = synth.make_pair(**cfg)
    grid_np = X.sampling_grid(wl["n_tilt"])
    grid = [(float(r["t"]), float(r["phi"])) for r in grid_np]
    pa = X.plan_image(case.A.shape[1], case.A.shape[0], grid_np, wl["n_levels"], 1.2, wl["n_features"], wl["fast"])
    pb = X.plan_image(case.B.shape[1], case.B.shape[0], grid_np, wl["n_levels"], 1.2, wl["n_features"], wl["fast"])
    A = torch.from_numpy(np.ascontiguousarray(case.A)).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(case.B)).to(dev)
    pattern = torch.from_numpy(synth.brief_pattern()).to(dev)
    run = X.BatchRunner([(case.A, np.ascontiguousarray(case.B))], grid, (1.0,), n_levels=wl["n_levels"],
                        n_features=wl["n_features"], fast_threshold=wl["fast"], device=dev,
                        queries_per_lane=args.matcher_q or "auto")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        run.run(pattern)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        run.run(pattern)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    ev_ms = ev0.elapsed_time(ev1) / args.steps

    # quality of the result (outside the timed region)
    pr = run.precision(0, case.H, 2.0).cpu().numpy()
    best = run.best[0].cpu().numpy().tolist()
    nv = len(grid)
    count_a = run.count[:nv].cpu().numpy().astype(np.int64)
    count_b = run.count[nv:2 * nv].cpu().numpy().astype(np.int64)
    comparisons = int(count_a.sum() * count_b.sum())

    # stage breakdown and the dominant kernel, each timed with HIP events on the launch stream
    st = X.StageRunner(pa, pb, dev)
    L = X.lib()

    def match_stage():
        # the matcher exactly as the timed step runs it: the batch's match plan on its descriptors
        X._check(L.xa_match_groups(run.mplan.host_ptr(), X._ptr(run.mplan.device(dev)), X._ptr(run.desc),
                                   X._ptr(run.count), run.n_views, 4, 5, X._ptr(run.matches), X._ptr(run.pair_count),
                                   X._ptr(run.best), X._stream()))

    stages = {"simulate": lambda: (st.simulate("a", A), st.simulate("b", B)),
              "extract": lambda: (st.extract("a", pattern), st.extract("b", pattern)),
              "match": match_stage}
    for f in stages.values():
        f()
    torch.cuda.synchronize()
    stage_ms = {}
    reps = max(3, args.steps)
    for name, f in stages.items():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            f()
        e1.record(stream)
        torch.cuda.synchronize()
        stage_ms[name] = e0.elapsed_time(e1) / reps
    st.match(4, 5)
    torch.cuda.synchronize()
    assert torch.equal(st.pair_count, run.pair_count), "stage-by-stage run disagrees with the batched entry"

    # the matcher (xa_match_groups = a counter fill, the matching kernel, a one-block argmax per group)
    match_s = stage_ms["match"] / 1e3
    # descriptor sets read once + the match records and counts written
    n_pairs = pa.n_views * pb.n_views
    algo_bytes = (pa.n_views + pb.n_views) * wl["n_features"] * 32 + n_pairs * wl["n_features"] * 8 + n_pairs * 4
    q = run.mplan_q
    if q in (MATCH_MATRIX, MATCH_MATRIX_PACKED):
        achieved = comparisons * MX_FLOPS_PER_CMP / match_s
        packed = ", query tiles packed across views" if q == MATCH_MATRIX_PACKED else ""
        head = {"kernel": f"k_match_mx (xa_match_groups, fp4 matrix-core contraction of +-1 descriptors{packed})",
                "bound": "mfma", "achieved": achieved / 1e12, "peak": FP4_PEAK_FLOPS / 1e12, "unit": "TFLOP/s",
                "frac": achieved / FP4_PEAK_FLOPS, "algorithmic_flops_per_launch": comparisons * MX_FLOPS_PER_CMP}
    else:
        achieved = comparisons * HAMMING_OPS_PER_CMP / match_s
        head = {"kernel": f"k_match<{q}> (xa_match_groups, popcount, {q} queries per lane)",
                "bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_OPS, "algorithmic_ops_per_launch": comparisons * HAMMING_OPS_PER_CMP}
    matcher = dict(head, **{
        "traffic": k_match_traffic(q),
        "traffic_unit": "bytes per launch (HBM, counter-measured)",
        "algorithmic_bytes_per_launch": algo_bytes,
        "comparisons_per_launch": comparisons,
        "comparisons_per_s": comparisons / match_s,
    })

    # warp: algorithmic bytes of the simulate stage (source read once per view, canvas + mask written)
    sim_bytes = 0
    for p in (pa, pb):
        h = p.header
        src = int(h["src_w"]) * int(h["src_h"])
        for v in p.views:
            sim_bytes += (4 * src if v["sigma"] > 0 else src) + 2 * int(v["width"]) * int(v["height"])
    n_views = pa.n_views + pb.n_views
    roofline = warp_roofline(case, grid_np, wl, dev, stream, pattern, match_stage)
    del st
    value = 1e3 / ms_per_step
    out = {
        "metric": "image pairs/s, full parameter-search path (simulate 45 views per image, ORB, 45x45 "
                  "all-view-pair Hamming match, best pair)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("u8 images, fp32 blur and warp, int32/int64 ORB, Hamming matching as an exact fp4 (+-1) "
                  "MFMA contraction with fp32 accumulation" if q in (MATCH_MATRIX, MATCH_MATRIX_PACKED) else
                  "u8 images, fp32 blur and warp, int32/int64 ORB, int32 popcount Hamming matching"),
        "data": "synthetic (seeded scene renderer; ground-truth affine pair)",
        "config": {
            "workload": f"{args.workload}: one {case.A.shape[1]}x{case.A.shape[0]} / {case.B.shape[1]}x{case.B.shape[0]} "
                        f"pair, B = A under tilt {cfg['t']} and rotation {math.degrees(cfg['psi']):.0f} deg",
            "views_per_image": len(grid), "n_levels": wl["n_levels"], "n_features": wl["n_features"],
            "fast_threshold": wl["fast"], "ratio": "4/5", "view_pairs": len(grid) ** 2,
            "parallelism": "single GPU",
        },
        "event_ms_per_step": ev_ms,
        "views_per_s": n_views * value,
        "stage_ms": stage_ms,
        "roofline": roofline,
        "matcher": matcher,
        "simulate_GBps": sim_bytes / (stage_ms["simulate"] / 1e3) / 1e9,
        "simulate_frac_hbm": sim_bytes / (stage_ms["simulate"] / 1e3) / HBM_PEAK_BPS,
        "best_pair": best,
        "precision_best_pair": {"correct": int(pr[0]), "matches": int(pr[1]), "th_px": 2.0},
        "keypoints": {"a": int(count_a.sum()), "b": int(count_b.sum())},
        "matcher_autotune": run.autotune,
        "warp_tiles": {"widths_per_class": [int(w) for w in tile_widths],
                       "rule": [16, 16, 8, 8, 8, 8, 4, 4],
                       "ms_per_class_and_candidate": None if tile_ms is None else np.round(tile_ms, 4).tolist(),
                       "candidates": list(X.WARP_CANDIDATES),
                       "tuner": ("fixed by --warp-tiles" if args.warp_tiles is not None else
                                 "built-in rule (--no-tune-tiles)" if tile_ms is None else
                                 "xa_tune_warp_tiles on a 1024x768 test image, class k = tilt sqrt(2)^k")},
        "blur_rows": {"rows_per_class": [int(r) for r in blur_rows], "default": 8,
                      "ms_per_class_4_8": None if blur_ms is None else np.round(blur_ms, 4).tolist(),
                      "tuner": ("fixed by --blur-rows" if args.blur_rows is not None else
                                "default (--no-tune-tiles)" if blur_ms is None else
                                "xa_tune_blur_rows on a 1024x768 test image, class k = tilt sqrt(2)^k")},
        "device": torch.cuda.get_device_name(0),
        "host_cpu": platform.processor() or platform.machine(),
        "host_cores": os.cpu_count(),
    }
    del run
    if args.batch_pairs > 0:
        out["batched"] = batched_leg(args, dev, pattern, raw, gen_s)
    if args.crops > 0:
        out["diffwarp"] = diffwarp_leg(args, dev)
    if args.l2_n > 0:
        out["l2_matcher"] = l2_leg(args, dev)
    if not args.no_sift:
        out["sift"] = sift_leg(args, dev)
    if not args.no_sweep:
        out["sweep"] = sweep_leg(args, dev, pattern)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
