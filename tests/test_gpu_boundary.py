"""GPU: boundary behaviour of the C ABI that needs a device (xa_check on a healthy stream)."""
import sys

import numpy as np
import pytest

import synth
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


def test_check_healthy_stream(dev):
    print("case: xa_check before, during and after a pair run, and after a host-rejected call", flush=True)
    sys.stdout.flush()
    L = X.lib()
    assert L.xa_check(X._stream()) == X.XA_OK
    case = synth.make_pair(**synth.PAIR_CONFIGS["tiny"])
    params = X.make_params([(t, f) for t, f in OP.sampling_grid(2)])
    pa = X.plan_image(256, 256, params, 3, 1.2, 300, 20)
    pb = X.plan_image(case.B.shape[1], case.B.shape[0], params, 3, 1.2, 300, 20)
    run = X.PairRunner(pa, pb, dev)
    run.run(torch.from_numpy(case.A).to(dev), torch.from_numpy(np.ascontiguousarray(case.B)).to(dev),
            torch.from_numpy(synth.brief_pattern()).to(dev))
    # work may still be running: the call does not wait and reports no error
    assert L.xa_check(X._stream()) == X.XA_OK
    torch.cuda.synchronize()
    assert L.xa_check(X._stream()) == X.XA_OK and L.xa_check(None) == X.XA_OK
    assert L.xa_match_views(256, 256, 0, 256, 256, 1, 100, 4, 5, 256, 256, 256, None) == X.XA_EINVAL
    assert L.xa_check(X._stream()) == X.XA_OK
    assert int(run.best[3].item()) > 0
