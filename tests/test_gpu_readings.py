"""The library's Lloyd stop on the exact 1-D instance the oracle's stopping
rule is pinned with (Section 5: relative tolerance, at most max_iter
updates): every centre and objective along the trace is an integer, so the
FP32 path must reproduce the exact trace and stop at the same update."""

import numpy as np
import pytest

from tests.gpu_common import require_gpu, say, to_dev
from tests.test_oracle_readings import LINE_C0, LINE_X, _exact_lloyd_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.mark.parametrize("tol,cap,iters", [
    (10.0, 300, 1), (0.5, 300, 3), (0.15, 300, 3), (0.1, 300, 5), (0.0, 300, 5),
    (45 / 314, 300, 3), (0.0, 0, 0), (0.0, 2, 2), (0.0, 4, 4),
])
def test_lloyd_stop_on_exact_trace(dev, tol, cap, iters):
    from paper_2403_18766_amd import api
    say("lloyd stop", tol, cap)
    trace, cents = _exact_lloyd_trace(LINE_X, LINE_C0, 5)
    S = to_dev(np.array(LINE_X, np.float32)[:, None], dev)
    C0 = to_dev(np.array(LINE_C0, np.float32)[:, None], dev)
    g = api.lloyd(S, C0, max_iter=cap, tol=tol)
    assert g["iters"] == iters
    assert g["f"] == float(trace[iters])
    assert np.array_equal(g["C"].cpu().numpy()[:, 0], np.array([float(c) for c in cents[iters]],
                                                               np.float32))
