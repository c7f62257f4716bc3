"""Size limits of the Lloyd path on the GPU: the largest k the LDS check
admits runs (narrow points: centroids, norms, fixed-point sums and the
kernel's own LDS fit one compute unit; wide points: the update's label
changes sorted by cluster), and the next k is refused with BM_E_ARG before
any launch."""

import numpy as np
import pytest

from paper_2403_18766_amd import datagen
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _admitted(api, S, C):
    from paper_2403_18766_amd._lib import BM_E_ARG
    try:
        return api.lloyd(S, C, max_iter=3)
    except api.BigmeansError as e:
        assert e.code == BM_E_ARG, str(e)
        return None


@pytest.mark.parametrize("n", [64, 61, 28, 4])
def test_largest_admitted_k_runs(dev, n):
    from paper_2403_18766_amd import api
    X = datagen.noisy_mixture(8_000, n, 20, seed=n)
    S = to_dev(X, dev)
    lo, hi = 1, 8_001     # admitted, refused (k <= s)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        ok = _admitted(api, S, to_dev(np.ascontiguousarray(X[:mid]), dev)) is not None
        lo, hi = (mid, hi) if ok else (lo, mid)
    say("n", n, "largest k", lo)
    assert 100 <= lo < 8_000
    g = _admitted(api, S, to_dev(np.ascontiguousarray(X[:lo]), dev))
    assert g is not None and np.isfinite(g["f"])
    assert _admitted(api, S, to_dev(np.ascontiguousarray(X[:lo + 1]), dev)) is None
    # the objective (no sums in LDS) accepts the same k
    f, _, _ = api.objective(S, to_dev(np.ascontiguousarray(X[:lo]), dev))
    assert np.isfinite(f)


def test_largest_admitted_k_runs_wide(dev):
    # 32,772 + 12 k bytes of the wide update within 160 KiB: k = 10,922
    from paper_2403_18766_amd import api
    X = datagen.noisy_mixture(11_500, 96, 20, seed=9)
    S = to_dev(X, dev)
    lo = 10_922
    say("wide n 96 largest k", lo)
    g = _admitted(api, S, to_dev(np.ascontiguousarray(X[:lo]), dev))
    assert g is not None and np.isfinite(g["f"])
    assert _admitted(api, S, to_dev(np.ascontiguousarray(X[:lo + 1]), dev)) is None
