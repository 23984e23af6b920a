"""GPU: the batched workload at its own sizes, checked against the oracle on samples it computes in
seconds.

Workload: the first 8 of the benchmark's 64 pairs (sides 480..2048, aspect 0.6..1.6, B under an
absolute tilt of 0..80 deg, seeds 3000..3007), the 45-view grid at scales {1, 0.5} (90 views per
image, 1440 views in all), 8 levels at 1.2, 500 keypoints per view, FAST threshold 20, ratio 4/5,
the matcher variant picked by the autotuner, views in the memory-bounded chunks of the default
workspace budget, run once eagerly and then as the captured graph the benchmark replays.

- Graph replays equal the eager run, byte for byte.
- The eager run equals the stand-alone stages (scale; simulate and extract chunk by chunk; group
  matching).
- Scaled sources of three pairs against the oracle's scale stage.
- Views of both scales and both images against the oracle's simulation of the oracle's source.
- ORB bit-exact on the GPU's own level-0 views of two views.
- Matching bit-exact on sampled view pairs of four pairs, each pair's best among them.
- Each pair's best is the argmax of its 8100 counts."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import match as OM
from oracle import orb as OO
from oracle import plan as OP
from oracle import simulate as OS

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu

N, LEVELS, FAST_T, N_PAIRS = 500, 8, 20, 8
SCALES = (1.0, 0.5)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batched(dev):
    t0 = time.time()
    say(f"case: first {N_PAIRS} pairs of the batched workload, 45-view grid at scales 1 and 0.5, 500 keypoints")
    cases = [synth.batch_pairs(1, seed=3000 + k)[0] for k in range(N_PAIRS)]
    pairs = [(c.A, np.ascontiguousarray(c.B)) for c in cases]
    for k, (A, B) in enumerate(pairs):
        say(f"[batched] pair {k}: A {A.shape[1]}x{A.shape[0]}, B {B.shape[1]}x{B.shape[0]}, "
            f"t = {cases[k].meta['t']:.2f}")
    say(f"[batched] generated in {time.time() - t0:.1f} s")
    grid = [(float(r["t"]), float(r["phi"])) for r in X.sampling_grid(5)]
    pattern_np = synth.brief_pattern()
    pattern = torch.from_numpy(pattern_np).to(dev)
    run = X.BatchRunner(pairs, grid, SCALES, n_levels=LEVELS, n_features=N, fast_threshold=FAST_T, device=dev,
                        queries_per_lane="auto")
    src0 = run.sources.clone()
    run.run(pattern)
    torch.cuda.synchronize()
    say(f"[batched] eager run: {run.n_views} views, {run.mplan.total_pairs} view pairs, "
        f"matcher variant {run.mplan_q}")
    eager = [t.clone() for t in (run.kp, run.desc, run.count, run.matches, run.pair_count, run.best)]
    # the stages chunk by chunk (the batch's memory-bounded chunks hold whole pairs, in order)
    buf = src0
    X.scale_sources(run.splan, buf)
    outs, arenas, masks = [], [], []
    for c in run.chunks:
        arena, mask = X.simulate_views(c, buf)
        outs.append(X.extract_orb(c, arena, mask, pattern))
        arenas.append(arena.cpu().numpy())
        masks.append(mask.cpu().numpy())
        del arena, mask
    kp, desc, count = (torch.cat([o[q] for o in outs]) for q in range(3))
    m, pc, best = X.match_groups(run.mplan, desc, count)
    torch.cuda.synchronize()
    say(f"[batched] stages over {len(run.chunks)} chunks done after {time.time() - t0:.1f} s")
    starts = np.cumsum([0] + [c.n_views for c in run.chunks])
    assert starts[-1] == run.n_views
    return dict(pairs=pairs, grid=grid, pattern=pattern, pattern_np=pattern_np, run=run, eager=eager,
                stages=(kp, desc, count, m, pc, best), buf=buf.cpu().numpy(), arenas=arenas, masks=masks,
                starts=starts)


def _level0(batched, vi):
    """Level 0 of global view vi (u8, mask) from its chunk's arena, and its view descriptor."""
    c = int(np.searchsorted(batched["starts"], vi, side="right")) - 1
    plan = batched["run"].chunks[c]
    li = vi - int(batched["starts"][c])
    return (plan.level_image(batched["arenas"][c], li, 0), plan.level_image(batched["masks"][c], li, 0).astype(bool),
            plan.views[li])


def test_batched_graph_replays_equal_the_eager_run(batched):
    run = batched["run"]
    run.capture(batched["pattern"])
    for rep in range(2):
        # outputs written in full on every run start from a sentinel, so a replay that did not
        # write them fails
        for t in (run.count, run.pair_count, run.best):
            t.fill_(-7)
        run.replay()
        torch.cuda.synchronize()
        for name, a, b in zip(("kp", "desc", "count", "matches", "pair_count", "best"),
                              (run.kp, run.desc, run.count, run.matches, run.pair_count, run.best), batched["eager"]):
            assert torch.equal(a, b), (rep, name)
        torch.cuda.synchronize()
    run.close()
    say("[batched] two graph replays equal the eager run")


def test_batched_eager_equals_stages(batched):
    for name, a, b in zip(("kp", "desc", "count", "matches", "pair_count", "best"), batched["eager"],
                          batched["stages"]):
        assert torch.equal(a, b), name
    c = batched["eager"][2].cpu().numpy()
    say(f"[batched] eager == stages; keypoints {int(c.sum())} (min {c.min()}, max {c.max()} per view)")


def _view_index(run, g, side, k, i, n_grid):
    a0, na, b0, nb = run.pair_views[g]
    return (a0 if side == "a" else b0) + k * n_grid + i


def _source_index(g, side, k):
    """Source arena order: per pair, A at each scale, then B at each scale."""
    return g * 2 * len(SCALES) + (0 if side == "a" else len(SCALES)) + k


@pytest.mark.parametrize("g,side", [(0, "a"), (3, "b"), (6, "a")])
def test_batched_scaled_sources(batched, g, side):
    img = batched["pairs"][g][0 if side == "a" else 1]
    _, U = OS.scale_image(img, 0.5)
    gs = batched["run"].arena.view(batched["buf"], _source_index(g, side, 1))
    assert gs.shape == U.shape
    du = np.abs(gs.astype(np.int64) - U.astype(np.int64))
    n_bad = int((du > 0).sum())
    assert du.max() <= 1 and n_bad <= max(1, 1e-4 * du.size), (g, side)
    say(f"[batched scale pair {g} {side}] {U.shape[1]}x{U.shape[0]}: u8 mismatches {n_bad}/{du.size}")


def _pick(grid, t, j):
    return [i for i, (ti, _) in enumerate(grid) if abs(ti - t) < 1e-9][j]


# (pair, image, scale index, tilt, j-th longitude at that tilt)
VIEW_CASES = [(1, "a", 0, 4.0, 3), (2, "b", 1, 2.0, 1), (5, "a", 1, 4 * 2 ** 0.5, 7), (7, "b", 0, 2 * 2 ** 0.5, 2)]


@pytest.mark.parametrize("g,side,k,t,j", VIEW_CASES)
def test_batched_views_against_the_oracle(batched, g, side, k, t, j):
    grid, run = batched["grid"], batched["run"]
    i = _pick(grid, t, j)
    img = batched["pairs"][g][0 if side == "a" else 1]
    src = img if SCALES[k] == 1.0 else OS.scale_image(img, SCALES[k])[1]
    ti, phi = grid[i]
    v = OP.plan_view(src.shape[1], src.shape[0], ti, phi, 0.0, 1.0)
    say(f"case: batched view pair {g} {side} s={SCALES[k]} t={ti:.3f} phi={np.degrees(phi):.1f} "
        f"({v.width}x{v.height})")
    V, M, U = OS.simulate_view(src, v)
    vi = _view_index(run, g, side, k, i, len(grid))
    gu, gm, _ = _level0(batched, vi)
    assert gu.shape == U.shape
    px, py = OS.view_coords(v)
    edge = (np.minimum(np.abs(px + 0.5), np.abs(px - (v.src_w - 0.5))) < 1e-9) | \
           (np.minimum(np.abs(py + 0.5), np.abs(py - (v.src_h - 0.5))) < 1e-9)
    assert np.all((gm == M) | edge)
    both = gm & M
    du = np.abs(gu[both].astype(np.int64) - U[both].astype(np.int64))
    assert du.max(initial=0) <= 1
    n_bad, n_px = int((du > 0).sum()), int(both.sum())
    assert n_bad <= max(1, 1e-4 * n_px)
    assert np.all(gu[~gm] == 0)
    say(f"[batched view {vi}] u8 mismatches {n_bad}/{n_px}")


@pytest.mark.parametrize("g,side,k,t,j", [(4, "a", 0, 2.0, 0), (0, "b", 1, 1.0, 0)])
def test_batched_orb_on_the_gpu_views(batched, g, side, k, t, j):
    grid, run = batched["grid"], batched["run"]
    vi = _view_index(run, g, side, k, _pick(grid, t, j), len(grid))
    U, M, vd = _level0(batched, vi)
    U = U.copy()
    say(f"case: batched ORB on view {vi} ({int(vd['width'])}x{int(vd['height'])})")
    dims = OP.level_dims(int(vd["width"]), int(vd["height"]), LEVELS)
    f = OO.extract_view(U, M, dims, OP.level_quotas(N, LEVELS), FAST_T, batched["pattern_np"])
    n = len(f["x"])
    kp, desc, count = batched["eager"][:3]
    g_kp = X.keypoints_np(kp)[vi][:n]
    assert int(count[vi]) == n
    for key in ("x", "y", "level", "harris", "bin"):
        assert np.array_equal(g_kp[key], f[key]), key
    assert np.array_equal(desc[vi].cpu().numpy()[:n], f["desc"])
    say(f"[batched ORB {vi}] {n} keypoints exact")


def test_batched_matching_on_sampled_pairs(batched):
    run = batched["run"]
    kp, desc, count, matches, pair_count, best = batched["eager"]
    c = count.cpu().numpy()
    d = desc.cpu().numpy()
    pc = pair_count.cpu().numpy()
    rng = np.random.default_rng(23)
    checked = 0
    for g in (0, 2, 5, 7):
        a0, na, b0, nb = run.pair_views[g]
        base = int(run.mplan.groups[g]["pair_base"])
        kb = int(np.argmax(pc[base:base + na * nb]))
        sample = {(kb // nb, kb % nb)} | {(int(a), int(b)) for a, b in rng.integers(0, [na, nb], (2, 2))}
        for a, b in sorted(sample):
            res, counts, _ = OM.match_views([d[a0 + a][:c[a0 + a]]], [d[b0 + b][:c[b0 + b]]], 4, 5)
            idx, d1, d2, _ = res[0]
            k = base + a * nb + b
            nq = int(c[a0 + a])
            m = X.matches_np(matches[k:k + 1])[0]
            assert np.array_equal(m[:nq]["t"], idx) and np.array_equal(m[:nq]["d1"], d1), (g, a, b)
            assert np.array_equal(m[:nq]["d2"], d2), (g, a, b)
            assert pc[k] == counts[0], (g, a, b)
            checked += 1
    say(f"[batched matching] exact on {checked} sampled view pairs of pairs 0, 2, 5, 7")


def test_batched_best_pair_is_the_argmax(batched):
    run = batched["run"]
    pc = batched["eager"][4].cpu().numpy()
    best = batched["eager"][5].cpu().numpy()
    for g in range(N_PAIRS):
        a0, na, b0, nb = run.pair_views[g]
        base = int(run.mplan.groups[g]["pair_base"])
        k = int(np.argmax(pc[base:base + na * nb]))
        assert best[g].tolist() == [k, k // nb, k % nb, int(pc[base + k])], g      # k within the pair
    say(f"[batched best] per pair: {[int(b[3]) for b in best]}")
