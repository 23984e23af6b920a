"""GPU: group matching and the batched path (many image pairs, original and scaled
sources, one call or one graph replay).

Group matching is exact against the oracle's matcher.  The batch is checked against
the single-pair entry point (same kernels, same inputs: identical bytes) and against
the stand-alone stages run one by one; its end result on scaled sources is compared
with the oracle's pipeline the way the single-pair test does it (the quantised views
may differ by a gray level on a few pixels, so counts are close rather than equal)."""
import sys

import numpy as np
import pytest

import synth
from oracle import match as OM
from oracle import pipeline as OPL
from oracle import plan as OP

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X.lib()
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pairs():
    out = []
    for (w, h, seed, t, psi) in ((256, 256, 1, 2.0, 30.0), (200, 160, 5, 1.6, -20.0), (96, 130, 7, 2.5, 60.0)):
        out.append(synth.make_pair(w, h, max(8, w * h // 1600), max(6, w * h // 2200), seed, t, 0.0,
                                   np.radians(psi)))
    return out


@pytest.mark.parametrize("q", [0, X.MATCH_MATRIX, X.MATCH_MATRIX_PACKED])
def test_match_groups_exact_random(dev, q):
    say(f"case: group matching of random descriptors, 4 groups with ragged sizes and an empty one (variant {q})")
    g = np.random.default_rng(31)
    N = 600
    sizes = [300, 17, 0, 600, 1, 256, 599, 64, 2, 450]
    D = np.zeros((len(sizes), N, 32), np.uint8)
    C = np.array(sizes, np.int32)
    descs = []
    for v, n in enumerate(sizes):
        d = g.integers(0, 256, (n, 32)).astype(np.uint8)
        D[v, :n] = d
        descs.append(d)
    descs[3][:200] = descs[0][:200] ^ np.uint8(4)
    D[3, :200] = descs[3][:200]
    groups = [(0, 3, 3, 4, 0), (5, 2, 0, 5, 12), (9, 0, 1, 3, 22), (2, 4, 6, 4, 22)]
    mp = X.plan_matches(np.array(groups, X.GROUP_DTYPE), N, q)
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    m, pc, best = X.match_groups(mp, t(D), t(C))
    torch.cuda.synchronize()
    m, pc, best = X.matches_np(m), pc.cpu().numpy(), best.cpu().numpy()
    for gi, (a0, na, b0, nb, base) in enumerate(groups):
        res, counts, rb = OM.match_views(descs[a0:a0 + na], descs[b0:b0 + nb])
        for k, (idx, d1, d2, acc) in enumerate(res):
            nq = len(descs[a0 + k // nb])
            assert np.array_equal(m[base + k][:nq]["t"], idx), (gi, k)
            assert np.array_equal(m[base + k][:nq]["d1"], d1) and np.array_equal(m[base + k][:nq]["d2"], d2)
        assert np.array_equal(pc[base:base + na * nb], counts), gi
        assert tuple(best[gi].tolist()) == tuple(rb), (gi, best[gi], rb)
    say(f"[groups] exact on 4 groups, best {best.tolist()}")


@pytest.mark.parametrize("q", X.MATCH_VARIANTS)
def test_match_groups_variants_agree(dev, q):
    say(f"case: group matching, queries_per_lane={q} equals the oracle at N=1100 (duplicate train rows: "
        "equal distances go to the lowest index)")
    g = np.random.default_rng(32 + q)
    N = 1100
    sizes = [1100, 1099, 513, 0, 1024]
    D = np.zeros((len(sizes), N, 32), np.uint8)
    descs = []
    for v, n in enumerate(sizes):
        d = g.integers(0, 256, (n, 32)).astype(np.uint8)
        D[v, :n] = d
        descs.append(d)
    descs[4][:300] = descs[0][:300] ^ np.uint8(16)
    D[4, :300] = descs[4][:300]
    for v in (0, 2):                                  # exact duplicates among train rows
        descs[v][400:480] = descs[v][:80]
        D[v, 400:480] = descs[v][400:480]
    descs[1][:80] = descs[0][:80]                     # queries equal to duplicated train rows
    D[1, :80] = descs[1][:80]
    groups = [(0, 2, 2, 3, 0), (4, 1, 0, 2, 6)]
    mp = X.plan_matches(np.array(groups, X.GROUP_DTYPE), N, q)
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    m, pc, best = X.match_groups(mp, t(D), t(np.array(sizes, np.int32)))
    torch.cuda.synchronize()
    m, pc, best = X.matches_np(m), pc.cpu().numpy(), best.cpu().numpy()
    for gi, (a0, na, b0, nb, base) in enumerate(groups):
        res, counts, rb = OM.match_views(descs[a0:a0 + na], descs[b0:b0 + nb])
        for k, (idx, d1, d2, acc) in enumerate(res):
            nq = len(descs[a0 + k // nb])
            assert np.array_equal(m[base + k][:nq]["t"], idx) and np.array_equal(m[base + k][:nq]["d1"], d1)
            assert np.array_equal(m[base + k][:nq]["d2"], d2), (q, gi, k)
        assert np.array_equal(pc[base:base + na * nb], counts) and tuple(best[gi].tolist()) == tuple(rb)


@pytest.mark.parametrize("q", [X.MATCH_MATRIX, X.MATCH_MATRIX_PACKED])
def test_match_groups_many_query_views(dev, q):
    say(f"case: matrix matcher (variant {q}), a group of 1100 query views (past the 1024 views whose query tiles a "
        "block packs: one query view per block) and packed groups of 1024, 300 (block-wide count scans) "
        "and 256 views (one wave's scan), ragged counts, N = 64")
    g = np.random.default_rng(35)
    N = 64
    sizes = g.integers(0, N + 1, 1103)
    sizes[:6] = [0, 1, 64, 33, 32, 0]
    sizes[1100:] = [64, 7, 0]
    D = np.zeros((len(sizes), N, 32), np.uint8)
    descs = []
    for v, n in enumerate(sizes):
        d = g.integers(0, 256, (int(n), 32)).astype(np.uint8)
        D[v, :n] = d
        descs.append(d)
    descs[2][:20] = descs[1100][:20] ^ np.uint8(8)
    D[2, :20] = descs[2][:20]
    groups = [(0, 1100, 1100, 3, 0), (3, 1024, 1100, 2, 3300), (5, 256, 1100, 1, 5348), (7, 300, 1101, 2, 5604)]
    mp = X.plan_matches(np.array(groups, X.GROUP_DTYPE), N, q)
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    m, pc, best = X.match_groups(mp, t(D), t(sizes.astype(np.int32)))
    torch.cuda.synchronize()
    m, pc, best = X.matches_np(m), pc.cpu().numpy(), best.cpu().numpy()
    for gi, (a0, na, b0, nb, base) in enumerate(groups):
        res, counts, rb = OM.match_views(descs[a0:a0 + na], descs[b0:b0 + nb])
        for k, (idx, d1, d2, acc) in enumerate(res):
            nq = len(descs[a0 + k // nb])
            assert np.array_equal(m[base + k][:nq]["t"], idx) and np.array_equal(m[base + k][:nq]["d1"], d1)
            assert np.array_equal(m[base + k][:nq]["d2"], d2), (gi, k)
        assert np.array_equal(pc[base:base + na * nb], counts) and tuple(best[gi].tolist()) == tuple(rb), gi
    say(f"[many views] exact on {sum(na * nb for _, na, _, nb, _ in groups)} view pairs")


def _grid(n_tilt):
    return [(t, f) for t, f in OP.sampling_grid(n_tilt)]


def test_batch_equals_single_pair_calls(dev, pairs):
    """Three pairs of different sizes in one batch (scale 1 only): every output byte equals
    what xa_match_pair gives for that pair alone."""
    say("case: batch of 3 pairs vs xa_match_pair per pair (bit-identical)")
    grid = _grid(2)
    pat = torch.from_numpy(synth.brief_pattern()).to(dev)
    br = X.BatchRunner([(p.A, np.ascontiguousarray(p.B)) for p in pairs], grid, (1.0,), n_levels=3, n_features=300,
                       device=dev)
    br.run(pat)
    torch.cuda.synchronize()
    nv = len(grid)
    params = X.make_params(grid)
    for pi, p in enumerate(pairs):
        B = np.ascontiguousarray(p.B)
        pa = X.plan_image(p.A.shape[1], p.A.shape[0], params, 3, 1.2, 300, 20)
        pb = X.plan_image(B.shape[1], B.shape[0], params, 3, 1.2, 300, 20)
        run = X.PairRunner(pa, pb, dev)
        run.run(torch.from_numpy(p.A).to(dev), torch.from_numpy(B).to(dev), pat)
        torch.cuda.synchronize()
        a0, b0 = 2 * pi * nv, (2 * pi + 1) * nv
        assert torch.equal(br.kp[a0:a0 + nv], run.kp_a) and torch.equal(br.desc[a0:a0 + nv], run.desc_a)
        assert torch.equal(br.kp[b0:b0 + nv], run.kp_b) and torch.equal(br.desc[b0:b0 + nv], run.desc_b)
        assert torch.equal(br.count[a0:a0 + nv], run.count_a) and torch.equal(br.count[b0:b0 + nv], run.count_b)
        base = int(br.mplan.groups[pi]["pair_base"])
        assert torch.equal(br.matches[base:base + nv * nv], run.matches), pi
        assert torch.equal(br.pair_count[base:base + nv * nv], run.pair_count), pi
        assert torch.equal(br.best[pi], run.best), pi
        assert torch.equal(br.precision(pi, p.H), run.precision(p.H)), pi
        say(f"[batch] pair {pi} ({p.A.shape[1]}x{p.A.shape[0]}): identical, best {run.best.tolist()}")


def test_batch_equals_stages_with_scales(dev, pairs):
    """Sources at scales 1 and 0.5: the batch equals the stand-alone calls (scale stage,
    simulate, extract, group matching) made one after the other on the same buffers."""
    say("case: batch with scales {1, 0.5} vs the stages called one by one")
    grid = _grid(2)
    pat = torch.from_numpy(synth.brief_pattern()).to(dev)
    imgs = [(p.A, np.ascontiguousarray(p.B)) for p in pairs[:2]]
    br = X.BatchRunner(imgs, grid, (1.0, 0.5), n_levels=3, n_features=300, device=dev)
    src0 = br.sources.clone()
    br.run(pat)
    torch.cuda.synchronize()
    buf = src0.clone()
    X.scale_sources(br.splan, buf)
    assert torch.equal(buf, br.sources)
    assert len(br.chunks) == 1
    arena, mask = X.simulate_views(br.chunks[0], buf)
    kp, desc, count = X.extract_orb(br.chunks[0], arena, mask, pat)
    m, pc, best = X.match_groups(br.mplan, desc, count)
    torch.cuda.synchronize()
    assert torch.equal(kp, br.kp) and torch.equal(desc, br.desc) and torch.equal(count, br.count)
    assert torch.equal(m, br.matches) and torch.equal(pc, br.pair_count) and torch.equal(best, br.best)
    say(f"[batch/scales] stage-by-stage identical; best per pair {best.tolist()}")


def test_batch_chunks_give_the_same_result(dev, pairs):
    """The same batch run as one chunk and as one chunk per pair (a tiny workspace budget):
    identical outputs, and the chunked workspace is the largest pair's, not the sum."""
    say("case: batch of 3 pairs (scales 1 and 0.5) as 1 chunk vs 3 chunks")
    grid = _grid(2)
    pat = torch.from_numpy(synth.brief_pattern()).to(dev)
    imgs = [(p.A, np.ascontiguousarray(p.B)) for p in pairs]
    one = X.BatchRunner(imgs, grid, (1.0, 0.5), n_levels=3, n_features=300, device=dev)
    many = X.BatchRunner(imgs, grid, (1.0, 0.5), n_levels=3, n_features=300, device=dev, chunk_bytes=1)
    assert len(one.chunks) == 1 and len(many.chunks) == 3
    assert many.ws.numel() < one.ws.numel()
    one.run(pat)
    many.run(pat)
    torch.cuda.synchronize()
    for a, b in zip((one.kp, one.desc, one.count, one.matches, one.pair_count, one.best),
                    (many.kp, many.desc, many.count, many.matches, many.pair_count, many.best)):
        assert torch.equal(a, b)
    say(f"[chunks] identical; workspace {one.ws.numel() >> 20} MiB as one chunk, {many.ws.numel() >> 20} MiB in 3")


def test_batch_scaled_pair_vs_oracle(dev, pairs):
    """End to end on the 256x256 pair with scales {1, 0.5} against the oracle pipeline."""
    say("case: batch (scales 1 and 0.5) vs the oracle pipeline on the tiny pair")
    p = pairs[0]
    B = np.ascontiguousarray(p.B)
    grid = _grid(2)
    br = X.BatchRunner([(p.A, B)], grid, (1.0, 0.5), n_levels=3, n_features=300, device=dev)
    br.run(torch.from_numpy(synth.brief_pattern()).to(dev))
    torch.cuda.synchronize()
    opts = OPL.OrbOptions(n_levels=3, n_features=300)
    ref = OPL.match_pair(p.A, B, grid, grid, opts, synth.brief_pattern(), (1.0, 0.5), (1.0, 0.5))
    best = br.best[0].cpu().numpy()
    counts = br.pair_count.cpu().numpy()
    say(f"[batch/oracle] gpu best {best.tolist()} oracle best {ref['best']}")
    assert abs(int(best[3]) - int(ref["best"][3])) <= max(5, 0.1 * ref["best"][3])
    assert np.corrcoef(counts, ref["counts"])[0, 1] > 0.95
    # keypoints of views of the scaled sources map back to original-image coordinates
    kp = X.keypoints_np(br.kp)
    nv = len(grid)
    for v in (nv, nv + 3):                       # views of A at scale 0.5
        n = int(br.count[v])
        f = ref["feats_a"][v]
        xs, ys = OPL.keypoints_to_source(f, ref["views_a"][v], opts, 0.5)
        same = min(n, len(f["x"]))
        # where the view bytes agree the keypoints do too; compare the common prefix of equal positions
        eq = (kp[v][:same]["x"] == f["x"][:same]) & (kp[v][:same]["y"] == f["y"][:same]) & \
             (kp[v][:same]["level"] == f["level"][:same])
        assert eq.mean() > 0.9
        assert np.allclose(kp[v][:same]["xs"][eq], xs[:same][eq], atol=1e-9)
        assert np.allclose(kp[v][:same]["ys"][eq], ys[:same][eq], atol=1e-9)


def test_batch_graph_replays(dev, pairs):
    """A captured batch replayed three times, with eager torch work and host syncs between
    the replays (outputs cleared each time): every replay equals the eager run."""
    say("case: batch captured in a HIP graph, 3 replays with eager work between them")
    grid = _grid(1)
    pat = torch.from_numpy(synth.brief_pattern()).to(dev)
    imgs = [(p.A, np.ascontiguousarray(p.B)) for p in pairs]
    br = X.BatchRunner(imgs, grid, (1.0, 0.5), n_levels=3, n_features=200, device=dev, chunk_bytes=1)
    assert len(br.chunks) == 3
    br.run(pat)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (br.kp, br.desc, br.count, br.matches, br.pair_count, br.best)]
    br.capture(pat)
    try:
        for r in range(3):
            for t in (br.kp, br.desc, br.count, br.matches, br.pair_count, br.best):
                t.zero_()
            junk = torch.randn(1 << 20, device=dev).sum()      # unrelated eager work
            torch.cuda.synchronize()
            br.replay()
            torch.cuda.synchronize()
            got = (br.kp, br.desc, br.count, br.matches, br.pair_count, br.best)
            for a, b in zip(ref, got):
                assert torch.equal(a, b), r
            say(f"[graph] replay {r} identical (junk {float(junk):.1f})")
    finally:
        br.close()


def test_autotuner_picks_a_variant_and_caches_it(dev, pairs):
    """The library's matcher autotuner times every variant, keeps the winner per device and
    key, and a batch built with it gives the same bytes as batches with each fixed variant."""
    say("case: matcher autotuner (popcount kernel with 1 / 2 / 4 queries per lane, matrix-core kernel plain and "
        "packed) and its cache")
    grid = _grid(1)
    pat = torch.from_numpy(synth.brief_pattern()).to(dev)
    imgs = [(p.A, np.ascontiguousarray(p.B)) for p in pairs[:2]]
    auto = X.BatchRunner(imgs, grid, (1.0,), n_levels=3, n_features=700, device=dev, queries_per_lane="auto")
    auto.run(pat)                                          # tunes on its own descriptors, then runs
    torch.cuda.synchronize()
    q, ms = auto.autotune["queries_per_lane"], auto.autotune["ms"]
    V = set(X.MATCH_VARIANTS)
    assert q in V and set(ms) == V and all(v > 0 for v in ms.values()) and ms[q] == min(ms.values())
    assert auto.mplan_q == q
    q2, ms2 = X.autotune_queries_per_lane(auto.mplan.groups, 700, dev, auto.desc, auto.count)
    assert q2 == q and ms2 == ms                          # served from the library's cache
    q3, ms3 = X.autotune_queries_per_lane(auto.mplan.groups, 700, dev, auto.desc, auto.count, use_cache=False)
    assert q3 in V and set(ms3) == V and ms3 != ms        # timed again
    q4, ms4 = X.autotune_queries_per_lane(auto.mplan.groups, 700, dev, auto.desc, auto.count)
    assert (q4, ms4) == (q3, ms3)                         # the new timing replaced the entry
    qr, msr = X.autotune_queries_per_lane(auto.mplan.groups, 700, dev)   # random full descriptors
    assert qr in V and set(msr) == V
    for fixed in X.MATCH_VARIANTS:
        r = X.BatchRunner(imgs, grid, (1.0,), n_levels=3, n_features=700, device=dev, queries_per_lane=fixed)
        r.run(pat)
        torch.cuda.synchronize()
        assert torch.equal(r.matches, auto.matches) and torch.equal(r.best, auto.best)
    say(f"[autotune] picked {q} queries per lane; ms {ms}")
