"""GPU: the full-size pair in the configuration the benchmark times, checked against the oracle on
samples it computes in seconds.

Workload: the 1024 x 768 / 725 x 725 synthetic pair, the 45-view grid of each image, 8 levels at
1.2, 1000 keypoints per view, FAST threshold 20, ratio 4/5, run by the batched entry point
(xa_match_batch) with the matrix-core matcher (the variant the autotuner picks).

- The batched run equals the stage-by-stage entry points on the same plans, byte for byte, at
  full size (so the samples below, taken from the stage buffers, are the batch's too).
- Views: four views of A and two of B against the oracle's simulation, to the tolerance of the
  small-size parity tests (among them the quarter turn at t = 4).
- ORB: bit-exact on the GPU's own level-0 views of three views.
- Matching: bit-exact on eight sampled view pairs of the GPU's descriptors, including the best.
- The best pair is the argmax of all 2025 pair counts, lowest index on ties."""
import sys

import numpy as np
import pytest

import synth
from oracle import match as OM
from oracle import orb as OO
from oracle import pipeline as OPL
from oracle import plan as OP
from oracle import simulate as OS

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu

N, LEVELS, FAST_T = 1000, 8, 20
WARP_TOL = 1e-4 * 255.0


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
def full(dev):
    say("case: full-size pair, batched entry (bench configuration) and stage-by-stage entries")
    case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
    grid_np = X.sampling_grid(5)
    grid = [(float(r["t"]), float(r["phi"])) for r in grid_np]
    B = np.ascontiguousarray(case.B)
    pattern_np = synth.brief_pattern()
    pattern = torch.from_numpy(pattern_np).to(dev)
    run = X.BatchRunner([(case.A, B)], grid, (1.0,), n_levels=LEVELS, n_features=N, fast_threshold=FAST_T,
                        device=dev, queries_per_lane=X.MATCH_MATRIX)
    run.run(pattern)
    pa = X.plan_image(case.A.shape[1], case.A.shape[0], grid_np, LEVELS, 1.2, N, FAST_T)
    pb = X.plan_image(B.shape[1], B.shape[0], grid_np, LEVELS, 1.2, N, FAST_T)
    st = X.StageRunner(pa, pb, dev)
    st.simulate("a", torch.from_numpy(np.ascontiguousarray(case.A)).to(dev))
    st.simulate("b", torch.from_numpy(B).to(dev))
    st.extract("a", pattern)
    st.extract("b", pattern)
    st.match(4, 5)
    torch.cuda.synchronize()
    return dict(case=case, B=B, grid=grid, pattern=pattern_np, run=run, st=st, pa=pa, pb=pb)


def test_full_batch_equals_stages(full):
    run, st = full["run"], full["st"]
    nv = full["pa"].n_views
    for key, sl in (("a", slice(0, nv)), ("b", slice(nv, 2 * nv))):
        s = st.side[key]
        assert torch.equal(run.count[sl], s["count"]), key
        assert torch.equal(run.kp[sl], s["kp"]) and torch.equal(run.desc[sl], s["desc"]), key
    assert torch.equal(run.pair_count, st.pair_count) and torch.equal(run.matches, st.matches)
    assert torch.equal(run.best[0], st.best)
    say(f"[full] batch == stages; best {st.best.tolist()}, keypoints {int(run.count.sum())}")


@pytest.mark.parametrize("q", [1, X.MATCH_MATRIX_PACKED])
def test_full_matcher_variants_agree(full, q):
    say(f"case: full-size pair, matcher variant {q} on the batch's own descriptors against the plain "
        "matrix-core kernel the batch ran")
    run = full["run"]
    mp = X.plan_matches(run.mplan.groups, N, q)
    m, pc, best = X.match_groups(mp, run.desc, run.count)
    torch.cuda.synchronize()
    assert torch.equal(m, run.matches) and torch.equal(pc, run.pair_count) and torch.equal(best, run.best)
    say(f"[full] variant {q}: identical matches, counts and best pair {best[0].tolist()}")


def _gpu_level0(plan, side, i):
    arena = side["arena"].cpu().numpy()
    mask = side["mask"].cpu().numpy()
    return plan.level_image(arena, i, 0).copy(), plan.level_image(mask, i, 0).astype(bool)


# view 25 is t = 4, phi = 90 deg: cos(phi) = 6e-17 puts a third of its source coordinates within
# 1e-11 below an integer, where the fp32 fraction rounds to 1
@pytest.mark.parametrize("key,i", [("a", 0), ("a", 20), ("a", 25), ("a", 44), ("b", 22), ("b", 25)])
def test_full_views_against_the_oracle(full, key, i):
    img = full["case"].A if key == "a" else full["B"]
    plan = full["pa"] if key == "a" else full["pb"]
    t, phi = full["grid"][i]
    v = OP.plan_view(img.shape[1], img.shape[0], t, phi, 0.0, 1.0)
    V, M, U = OS.simulate_view(img, v)
    gu, gm = _gpu_level0(plan, full["st"].side[key], i)
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
    say(f"[full view {key}{i}] {v.width}x{v.height}: u8 mismatches {n_bad}/{n_px}")


@pytest.mark.parametrize("key,i", [("a", 0), ("a", 44), ("b", 20)])
def test_full_orb_on_the_gpu_views(full, key, i):
    plan = full["pa"] if key == "a" else full["pb"]
    side = full["st"].side[key]
    U, M = _gpu_level0(plan, side, i)
    v = plan.views[i]
    dims = OP.level_dims(int(v["width"]), int(v["height"]), LEVELS)
    f = OO.extract_view(U, M, dims, OP.level_quotas(N, LEVELS), FAST_T, full["pattern"])
    n = len(f["x"])
    kp = X.keypoints_np(side["kp"])[i]
    assert int(side["count"][i]) == n
    g = kp[:n]
    for k in ("x", "y", "level", "harris", "bin"):
        assert np.array_equal(g[k], f[k]), k
    assert np.array_equal(side["desc"][i].cpu().numpy()[:n], f["desc"])
    img = full["case"].A if key == "a" else full["B"]
    t, phi = full["grid"][i]
    ov = OP.plan_view(img.shape[1], img.shape[0], t, phi, 0.0, 1.0)
    xs, ys = OPL.keypoints_to_source(f, ov, OPL.OrbOptions(n_levels=LEVELS, n_features=N))
    assert np.allclose(g["xs"], xs, atol=1e-9) and np.allclose(g["ys"], ys, atol=1e-9)
    say(f"[full ORB {key}{i}] {n} keypoints exact")


def test_full_matching_on_sampled_pairs(full):
    st = full["st"]
    na, nb = full["pa"].n_views, full["pb"].n_views
    best = st.best.tolist()
    rng = np.random.default_rng(7)
    pairs = {(int(best[1]), int(best[2]))} | {(int(a), int(b)) for a, b in rng.integers(0, [na, nb], (7, 2))}
    ca, cb = st.side["a"]["count"].cpu().numpy(), st.side["b"]["count"].cpu().numpy()
    da, db = st.side["a"]["desc"].cpu().numpy(), st.side["b"]["desc"].cpu().numpy()
    m = X.matches_np(st.matches)
    pc = st.pair_count.cpu().numpy()
    for a, b in sorted(pairs):
        res, counts, _ = OM.match_views([da[a][:ca[a]]], [db[b][:cb[b]]], 4, 5)
        idx, d1, d2, _ = res[0]
        k = a * nb + b
        nq = int(ca[a])
        assert np.array_equal(m[k][:nq]["t"], idx) and np.array_equal(m[k][:nq]["d1"], d1), (a, b)
        assert np.array_equal(m[k][:nq]["d2"], d2), (a, b)
        assert pc[k] == counts[0], (a, b)
    say(f"[full matching] exact on view pairs {sorted(pairs)}")


def test_full_best_pair_is_the_argmax(full):
    pc = full["st"].pair_count.cpu().numpy()
    best = full["st"].best.tolist()
    nb = full["pb"].n_views
    k = int(np.argmax(pc))                                     # first maximum: lowest index
    assert best == [k, k // nb, k % nb, int(pc[k])]
