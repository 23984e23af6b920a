"""GPU: the allocation-free L2 matcher (xa_match_l2_noalloc, library-owned scratch) against the
workspace entry xa_match_l2 on the same inputs, bit for bit, over consecutive calls that reuse the
scratch with a smaller input on the second call."""
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


def _to(dev, A):
    return torch.from_numpy(np.ascontiguousarray(A, np.uint8).reshape(-1, 128)).to(dev)


def _both(dev, Q, T, num, den):
    q, t = _to(dev, Q), _to(dev, T)
    ref_out, ref_cnt = X.match_l2(q, t, num, den)
    out = torch.empty((max(len(Q), 1), 3), dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    got_out, got_cnt = X.match_l2_noalloc(q, t, num, den, out=out, count=cnt)
    torch.cuda.synchronize()
    return (X.l2_matches_np(ref_out), int(ref_cnt.cpu()[0])), (X.l2_matches_np(got_out), int(got_cnt.cpu()[0]))


def _same(ref, got, label):
    (r, rc), (g, gc) = ref, got
    assert len(r) == len(g), label
    for f in ("t", "d1", "d2"):
        assert np.array_equal(r[f], g[f]), (label, f)
    assert rc == gc, label
    say(f"[{label}] {len(g)} queries identical, {gc} pass the ratio test")


def test_noalloc_equals_workspace_entry_on_consecutive_calls(dev):
    # first call: many queries over several train slices, so the scratch holds many partials;
    # second call: a smaller input on the same scratch, whose stale partials must not leak in
    say("case: noalloc 3000 x 9000 (ratio 3/4), then 300 x 517 (ratio 4/5) on the same scratch")
    Q1, T1, _ = synth.sift_like_sets(3000, 9000, 21)
    _same(*_both(dev, Q1, T1, 3, 4), "noalloc first call 3000 x 9000")
    Q2, T2, _ = synth.sift_like_sets(300, 517, 22)
    _same(*_both(dev, Q2, T2, 4, 5), "noalloc second call 300 x 517")
    say("case: noalloc 70 x 20000 (157 train slices), then 1 x 1 and 5 x 0")
    Q3, T3, _ = synth.sift_like_sets(70, 20000, 23)
    _same(*_both(dev, Q3, T3, 3, 4), "noalloc 70 x 20000")
    Q4, T4, _ = synth.sift_like_sets(1, 1, 24)
    _same(*_both(dev, Q4, T4, 3, 4), "noalloc 1 x 1")
    Q5 = synth.sift_like_descriptors(5, 25)
    _same(*_both(dev, Q5, np.zeros((0, 128), np.uint8), 3, 4), "noalloc 5 x 0")


def test_noalloc_rejects_counts_beyond_the_limit(dev):
    say("case: noalloc argument checks on the host (no kernel runs)")
    q = torch.zeros((1, 128), dtype=torch.uint8, device=dev)
    L = X.lib()
    st = L.xa_match_l2_noalloc(X._ptr(q), (1 << 20) + 1, X._ptr(q), 1, 3, 4, X._ptr(q), X._ptr(q), None)
    assert st == X.XA_EINVAL
    st = L.xa_match_l2_noalloc(X._ptr(q), 1, X._ptr(q), 1, 3, 0, X._ptr(q), X._ptr(q), None)
    assert st == X.XA_EINVAL
