"""GPU: the warp tile tuner (xa_tune_warp_tiles) and tuned plans.  The tuner times every
candidate width per compression class and returns valid widths; a plan made with tuned widths
(or any other widths) simulates the same views byte for byte as the rule's plan, since the
tile width changes only which threads compute a pixel, not how."""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
X = pytest.importorskip("paper_2503_03479_amd.xaffine")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X.lib()
    return torch.device("cuda:0")


def test_tuner_returns_valid_widths(dev):
    say("case: warp tile tuner on a 512 x 384 test image")
    try:
        widths, ms = X.tune_warp_tiles(dev, 512, 384, apply=False, cache=False)
        torch.cuda.synchronize()
        assert all(int(w) in X.WARP_CANDIDATES for w in widths)
        assert np.all(ms > 0) and np.all(np.isfinite(ms))
        # each class keeps the rule's width unless its fastest candidate beats it by more than 3 %
        rule = [16, 16, 8, 8, 8, 8, 4, 4]
        for k in range(X.WARP_CLASSES):
            t_rule = ms[k, X.WARP_CANDIDATES.index(rule[k])]
            best = int(np.argmin(ms[k]))
            want = X.WARP_CANDIDATES[best] if ms[k, best] < np.float32(0.97) * t_rule else rule[k]
            assert int(widths[k]) == want, (k, widths.tolist(), ms[k].tolist())
        say(f"[tuner] widths {widths.tolist()}")
    finally:
        X.set_warp_tiles(None)


def test_tuned_and_rule_plans_simulate_the_same_views(dev):
    say("case: the full-size pair's image A: rule widths against widths 64 / 4 / 32 per class")
    case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
    src = torch.from_numpy(np.ascontiguousarray(case.A)).to(dev)
    grid = X.sampling_grid(5)
    outs = []
    try:
        for widths in (None, [64, 4, 32, 4, 64, 16, 4, 4], [4, 64, 4, 32, 8, 64, 4, 4]):
            X.set_warp_tiles(widths)
            plan = X.plan_image(1024, 768, grid, 8, 1.2, 1000, 20)
            arena, mask = X.simulate_views(plan, src)
            torch.cuda.synchronize()
            outs.append((plan.views["warp_tile_w"].copy(), arena.cpu().numpy(), mask.cpu().numpy()))
    finally:
        X.set_warp_tiles(None)
    (w0, a0, m0) = outs[0]
    for (w, a, m) in outs[1:]:
        assert not np.array_equal(w, w0)
        assert np.array_equal(a, a0) and np.array_equal(m, m0)
    say("[tiles] views identical under three width tables")


def test_blur_rows_tuner_and_identical_blurs(dev):
    """The blur's outputs per thread (4 or 8) change only which thread makes a blurred sample: the
    blurred planes (fp32 values of the views) are bit-identical under three tables, and the tuner
    keeps 8 unless 4 is more than 3 % faster in a class."""
    say("case: blur rows tuner on 512 x 384; the full-size pair's image A under rows 8 / 4 / mixed")
    try:
        rows, ms = X.tune_blur_rows(dev, 512, 384, apply=False, cache=False)
        torch.cuda.synchronize()
        assert rows[0] == 8 and np.all(ms[0] == 0)
        for k in range(1, X.WARP_CLASSES):
            assert np.all(ms[k] > 0) and np.all(np.isfinite(ms[k]))
            want = 4 if ms[k, 0] < np.float32(0.97) * ms[k, 1] else 8
            assert int(rows[k]) == want, (k, rows.tolist(), ms[k].tolist())
        say(f"[blur rows] tuned {rows.tolist()}")
        case = synth.make_pair(**synth.PAIR_CONFIGS["full"])
        src = torch.from_numpy(np.ascontiguousarray(case.A)).to(dev)
        grid = X.sampling_grid(5)
        outs = []
        for table in (None, [4] * 8, [8, 4, 8, 4, 4, 8, 4, 8]):
            X.set_blur_rows(table)
            plan = X.plan_image(1024, 768, grid, 8, 1.2, 1000, 20)
            arena, mask, vals = X.simulate_views(plan, src, values=True)
            torch.cuda.synchronize()
            outs.append((plan.views["blur_rows"].copy(), vals.cpu().numpy(), arena.cpu().numpy()))
    finally:
        X.set_blur_rows(None)
    (r0, v0, a0) = outs[0]
    for (r, v, a) in outs[1:]:
        assert not np.array_equal(r, r0)
        assert np.array_equal(v, v0) and np.array_equal(a, a0)
    say("[blur rows] view values identical under three tables")
