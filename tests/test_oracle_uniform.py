"""Properties of the per-site uniforms (Sec. 3.2, Algorithm 1 "probs"; Sec. 5.1 random_uniform).

Each site gets its own 32-bit integer x, u = x / 2^32 in [0, 1).  Whatever the mapping from
Philox words to sites, a correct one makes the x of distinct (site, sweep, colour) distinct
and iid uniform: every bit balanced, bits uncorrelated with each other and across neighbours,
and P(x < T) = T / 2^32.  A mapping that reused a word, a bit position or a counter would
fail one of these.
"""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def sample(oracle_lib):
    xs = []
    rng = np.random.default_rng(7)
    for _ in range(2000):
        r = int(rng.integers(0, 4096))
        c0 = int(rng.integers(0, 64)) * 64
        t = int(rng.integers(0, 10**6))
        q = int(rng.integers(0, 2))
        # all 32 colour-q sites of one Philox group (64 consecutive columns of row r)
        row = [oracle_lib.uniform(3, r, c0 + 2 * j + ((r + q) & 1), t, q) for j in range(32)]
        xs.append(row)
    return np.array(xs, dtype=np.uint64)


def test_uniforms_distinct(sample):
    flat = sample.ravel()
    assert len(np.unique(flat)) >= flat.size - 2


def test_every_bit_balanced(sample):
    flat = sample.ravel()
    n = flat.size
    for b in range(32):
        ones = int(((flat >> np.uint64(b)) & np.uint64(1)).sum())
        assert abs(ones - n / 2) < 5 * math.sqrt(n / 4), b


def test_bits_uncorrelated(sample):
    flat = sample.ravel()
    bits = np.stack([((flat >> np.uint64(b)) & np.uint64(1)).astype(np.float64) for b in range(32)])
    corr = np.corrcoef(bits)
    off = corr[~np.eye(32, dtype=bool)]
    assert np.abs(off).max() < 5 / math.sqrt(flat.size)


def test_neighbouring_sites_uncorrelated(sample):
    a = sample[:, :-1].ravel().astype(np.float64)
    b = sample[:, 1:].ravel().astype(np.float64)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


def test_top_byte_uniform(sample):
    top = (sample.ravel() >> np.uint64(24)).astype(np.int64)
    counts = np.bincount(top, minlength=256)
    expected = top.size / 256
    chi2 = ((counts - expected) ** 2 / expected).sum()
    # 255 degrees of freedom: mean 255, sd ~22.6; 6 sd bound
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)


def test_acceptance_frequency(oracle_lib, sample):
    flat = sample.ravel()
    for beta in (0.2, 0.44068679350977147, 0.6):
        for T in oracle_lib.thresholds(beta):
            p = T / 2**32
            k = int((flat < T).sum())
            assert abs(k - p * flat.size) < 5 * math.sqrt(flat.size * p * (1 - p))


def test_uniform_depends_on_sweep_and_colour(oracle_lib):
    base = oracle_lib.uniform(1, 10, 21, 5, 1)
    assert base != oracle_lib.uniform(1, 10, 21, 6, 1)
    assert base != oracle_lib.uniform(2, 10, 21, 5, 1)
    assert base != oracle_lib.uniform(1, 12, 21, 5, 1)
    assert base != oracle_lib.uniform(1, 10, 21, 5, 0)


def test_colours_draw_independent_uniforms(oracle_lib):
    # The same site (r, c) with the same sweep index under the two colour labels: a counter that
    # dropped the colour would give equal uniforms, a shared word correlated ones.
    rng = np.random.default_rng(8)
    xs = []
    for _ in range(4000):
        r, c, t = int(rng.integers(0, 4096)), int(rng.integers(0, 4096)), int(rng.integers(0, 1 << 20))
        xs.append((oracle_lib.uniform(5, r, c, t, 0), oracle_lib.uniform(5, r, c, t, 1)))
    x = np.array(xs, dtype=np.float64)
    assert (x[:, 0] != x[:, 1]).all()
    corr = np.corrcoef(x[:, 0], x[:, 1])[0, 1]
    assert abs(corr) < 5 / math.sqrt(len(x))
