"""The seeded input generators (CPU): the shapes and distributions the
workload recipes state.  These inputs feed both the oracle and the GPU path,
so a generator that drifts from its recipe would make every parity test
compare the wrong workload."""

import numpy as np
import pytest
from scipy.special import ive

from paper_2403_18766_amd import datagen


def _mean_resultant(p, kappa):
    # E[x . mu] for vMF on S^(p-1): A_p(kappa) = I_{p/2}(kappa) / I_{p/2-1}(kappa)
    return ive(p / 2.0, kappa) / ive(p / 2.0 - 1.0, kappa)


@pytest.mark.parametrize("kappa", [60.0, 120.0, 200.0])
def test_vmf_cosines_follow_wood_sampler_mean(kappa):
    w = datagen._vmf_cosines(np.random.default_rng(0), kappa, 768, 100_000)
    assert np.all(np.abs(w) <= 1.0)
    se = w.std() / np.sqrt(w.size)
    assert abs(w.mean() - _mean_resultant(768, kappa)) < 5 * se


def test_vmf_cosines_low_dimension_against_closed_form():
    # on S^2 the cosine has density proportional to exp(kappa w) on [-1, 1]:
    # E[w] = coth(kappa) - 1 / kappa
    kappa = 3.0
    w = datagen._vmf_cosines(np.random.default_rng(1), kappa, 3, 200_000)
    want = 1.0 / np.tanh(kappa) - 1.0 / kappa
    assert abs(w.mean() - want) < 5 * w.std() / np.sqrt(w.size)


def test_vmf_mixture_device_recipe_on_cpu():
    torch = pytest.importorskip("torch")
    X = datagen.vmf_mixture_device(500, 64, 4, "cpu", seed=3).numpy()
    assert X.shape == (2_000, 64) and X.dtype == np.float32
    assert np.abs(np.linalg.norm(X.astype(np.float64), axis=1) - 1.0).max() < 1e-6
    # the same seed gives the same points
    Y = datagen.vmf_mixture_device(500, 64, 4, "cpu", seed=3).numpy()
    assert np.array_equal(X, Y)
    # the first cluster's mean direction is the first draw of default_rng(seed):
    # a quarter of the points sit at cosine ~ A_p(kappa) to it (kappa in
    # [50, 200]: 0.64 .. 0.95 for p = 64), the rest near 0 (spread 1/sqrt(p))
    mu = np.random.default_rng(3).standard_normal(64)
    mu /= np.linalg.norm(mu)
    cos = X.astype(np.float64) @ mu
    own = cos > 0.4
    assert own.sum() == 500
    assert _mean_resultant(64, 50.0) - 0.05 < cos[own].mean() < _mean_resultant(64, 200.0) + 0.05
