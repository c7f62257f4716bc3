"""bm_objective_noalloc (static workspace, no allocation) against bm_objective
through the C ABI: the same f bits, labels and near-tie counts, on two calls
in a row (the second smaller, so the static workspace still holds the first
call's larger contents), for narrow points, wide points on the FP32 and BF16
matrix cores, and a ragged tail; sizes beyond the static workspace are
refused on the host before any launch."""

import numpy as np
import pytest

from paper_2403_18766_amd import datagen
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _both(api, torch, X, C, prec):
    m = X.shape[0]
    f_ref, lab_ref, near_ref = api.objective(X, C, labels=True, near_ties=True, prec=prec)
    lab = torch.full((m,), -7, dtype=torch.int32, device=X.device)
    f, near = api.objective_noalloc(X, C, labels_out=lab, near_ties=True, prec=prec)
    return (f_ref, lab_ref.cpu().numpy(), near_ref), (f, lab.cpu().numpy(), near)


@pytest.mark.parametrize("n,k,prec,sizes", [
    (28, 50, 0, (300_001, 1_000)),       # narrow, several tiles, then a small ragged call
    (16, 200, 0, (50_000, 777)),         # many centres (wave-level re-decision)
    (96, 100, 0, (70_000, 513)),         # wide points, FP32 matrix cores
    (96, 160, 1, (40_000, 2_049)),       # wide points, BF16 matrix cores, two centre groups
])
def test_noalloc_objective_equals_objective(dev, n, k, prec, sizes):
    import torch

    from paper_2403_18766_amd import api
    Xh = datagen.noisy_mixture(max(sizes), n, 20, seed=n + k)
    Ch = np.ascontiguousarray(Xh[np.random.default_rng(k).choice(Xh.shape[0], k, replace=False)])
    C = to_dev(Ch, dev)
    for call, m in enumerate(sizes):
        say("noalloc objective", n, k, prec, "call", call, "m", m)
        X = to_dev(np.ascontiguousarray(Xh[:m]), dev)
        (f_ref, lab_ref, near_ref), (f, lab, near) = _both(api, torch, X, C, prec)
        assert f == f_ref
        assert np.array_equal(lab, lab_ref)
        assert near == near_ref


def test_noalloc_objective_without_outputs(dev):
    from paper_2403_18766_amd import api
    Xh = datagen.noisy_mixture(20_000, 12, 8, seed=1)
    X = to_dev(Xh, dev)
    C = to_dev(np.ascontiguousarray(Xh[:9]), dev)
    f_ref, _, _ = api.objective(X, C, labels=False, near_ties=False)
    f, near = api.objective_noalloc(X, C, near_ties=False)
    assert f == f_ref and near is None


def test_noalloc_objective_refuses_sizes_beyond_workspace(dev):
    # the host refuses before any launch: m claims far more rows than the
    # static workspace can cover (the rows themselves are never read)
    from paper_2403_18766_amd import _lib, api
    X = to_dev(datagen.noisy_mixture(1_000, 4, 3, seed=2), dev)
    C = to_dev(np.zeros((3, 4), np.float32), dev)
    lib, c = api._ctx(X.device)
    import ctypes as ct
    f = ct.c_double()
    rc = lib.bm_objective_noalloc(c, ct.c_void_p(X.data_ptr()), 1 << 40, 4,
                                  ct.c_void_p(C.data_ptr()), 3, 0, ct.byref(f), None, None)
    assert rc == _lib.BM_E_ARG
    assert b"static workspace" in lib.bm_strerror(c)
