"""Pins of the oracle's random-number contract (no GPU).

Philox4x64-10 is checked against numpy's independent implementation, the
SplitMix64 finaliser against published outputs, and the Feistel sampler by
exhaustive bijection checks and chi-square uniformity."""

import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle import rng


def _numpy_block(ctr, key):
    # numpy's Philox(counter=c) increments before its first block, so it emits B(c + 1).
    c = (sum(int(w) << (64 * i) for i, w in enumerate(ctr)) - 1) % (1 << 256)
    words = [(c >> (64 * i)) & rng.MASK64 for i in range(4)]
    g = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                         key=np.array(key, dtype=np.uint64))
    return tuple(int(v) for v in g.random_raw(4))


def test_philox_scalar_matches_numpy():
    r = np.random.default_rng(123)
    cases = [((0, 0, 0, 0), (0, 0)), ((1, 0, 0, 0), (0, 0)),
             ((0, 1, 0, 0), (5, 7)),                     # carry out of word 0 for numpy's c-1
             ((rng.MASK64, rng.MASK64, 0, 0), (1, 2)),
             ((3, 0, 0, 1), (rng.MASK64, rng.MASK64))]
    for _ in range(2000):
        ctr = tuple(int(v) for v in r.integers(0, 2**64, size=4, dtype=np.uint64))
        key = tuple(int(v) for v in r.integers(0, 2**64, size=2, dtype=np.uint64))
        cases.append((ctr, key))
    for ctr, key in cases:
        assert rng.philox_block_scalar(ctr, key) == _numpy_block(ctr, key)


def test_philox_vectorised_matches_scalar():
    r = np.random.default_rng(7)
    ctr = r.integers(0, 2**64, size=(4, 10_000), dtype=np.uint64)
    key = (0x0123456789ABCDEF, 0xFEDCBA9876543210)
    out = rng.philox_block(ctr[0], ctr[1], ctr[2], ctr[3], key)
    for i in range(0, 10_000, 97):
        ref = rng.philox_block_scalar(tuple(int(c[i]) for c in ctr), key)
        assert tuple(int(o[i]) for o in out) == ref


def test_mix64_published_outputs(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64.json")) as f:
        g = json.load(f)
    x = np.array([int(h, 16) for h in g["inputs_hex"]], dtype=np.uint64)
    got = [int(v) for v in rng.mix64(x)]
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_conversions():
    assert rng.u01(0) == 0.0
    assert rng.u01(rng.MASK64) == 1.0 - 2.0 ** -53
    assert rng.mulhi(rng.MASK64, 10) == 9
    assert rng.mulhi(0, 10) == 0
    assert rng.mulhi(1 << 63, 7) == 3


@pytest.mark.parametrize("m,h", [(1, 1), (2, 1), (4, 1), (5, 2), (16, 2), (17, 3),
                                 (1 << 20, 10), ((1 << 20) + 1, 11), (10_000_000, 12)])
def test_half_bits(m, h):
    assert rng.feistel_half_bits(m) == h
    assert 4 ** h >= m


def test_feistel_is_a_permutation_exhaustive():
    ms = list(range(1, 513)) + list(range(513, 4097, 37)) + [4096]
    for m in ms:
        for seed, worker, g in ((0, 0, 0), (11, 3, 17)):
            idx = rng.sample_indices(m, m, seed, worker, rng.PURPOSE_SAMPLE, g)
            assert np.array_equal(np.sort(idx), np.arange(m)), m


def test_feistel_raw_permutation_of_domain():
    for h in (1, 2, 5, 8):
        rk = rng.feistel_round_keys(rng.stream_key(9, 1, rng.PURPOSE_SAMPLE), 4)
        y = rng.feistel_permute(np.arange(4 ** h, dtype=np.uint64), h, rk)
        assert np.array_equal(np.sort(y.astype(np.int64)), np.arange(4 ** h))


def test_sample_prefix_property_and_range():
    # A sample of size s is the first s elements of the size-m ordering (sample order = i order).
    full = rng.sample_indices(1000, 1000, 5, 2, rng.PURPOSE_SAMPLE, 9)
    part = rng.sample_indices(1000, 137, 5, 2, rng.PURPOSE_SAMPLE, 9)
    assert np.array_equal(full[:137], part)
    assert len(np.unique(part)) == 137 and part.min() >= 0 and part.max() < 1000


def test_sample_inclusion_uniform_chi2():
    m, s, trials = 60, 20, 6000
    counts = np.zeros(m)
    first = np.zeros(m)
    for g in range(trials):
        idx = rng.sample_indices(m, s, 1, 0, rng.PURPOSE_SAMPLE, g)
        counts[idx] += 1
        first[idx[0]] += 1
    exp = trials * s / m
    chi = ((counts - exp) ** 2 / exp).sum()
    # counts are not independent across cells (fixed total); the statistic is a
    # conservative uniformity check at a 1e-4 level.
    assert stats.chi2.sf(chi, m - 1) > 1e-4
    expf = trials / m
    chif = ((first - expf) ** 2 / expf).sum()
    assert stats.chi2.sf(chif, m - 1) > 1e-4


def test_streams_differ_by_purpose_and_worker():
    a = rng.sample_indices(10_000, 50, 0, 0, rng.PURPOSE_SAMPLE, 0)
    b = rng.sample_indices(10_000, 50, 0, 0, rng.PURPOSE_RECALC, 0)
    c = rng.sample_indices(10_000, 50, 0, 1, rng.PURPOSE_SAMPLE, 0)
    d = rng.sample_indices(10_000, 50, 0, 0, rng.PURPOSE_SAMPLE, 1)
    assert not np.array_equal(a, b) and not np.array_equal(a, c) and not np.array_equal(a, d)
