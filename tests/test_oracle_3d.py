"""Pins of the oracle's three-dimensional chain (the d-dimensional hypercubic lattice of Sec. 3,
with the checkerboard colouring of Fig. 1 extended to three dimensions).

Each check is against something other than the oracle's own arithmetic: numpy neighbour sums
and bond sums, exact limits (beta = 0 flips every spin; zero temperature from the Neel state),
flip frequencies of constructed states where every site of a class has the same local field,
the Boltzmann distribution of the 2 x 2 x 2 torus by enumeration, high-precision thresholds,
and the full-lattice run for the light-cone block.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import exact as X
from paper_1903_11714_amd import analysis as A

Z_MAX = 4.5


def _roll_field(s):
    s = s.astype(np.int64)
    return sum(np.roll(s, k, axis=ax) for ax in (0, 1, 2) for k in (1, -1))


def _parity(L):
    z, y, x = np.indices((L, L, L))
    return (x + y + z) & 1


def _random(L, seed, p_down=0.5):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L, L)) < p_down, -1, 1).astype(np.int8)


@pytest.mark.parametrize("beta", [0.0, 0.1, 0.2216546, 0.35, 1.0, math.inf])
def test_thresholds3(oracle_lib, beta):
    T2, T4, T6 = oracle_lib.thresholds3(beta)
    # s = 2, 4 are the two-dimensional thresholds (pinned on their own)
    assert (T2, T4) == oracle_lib.thresholds(beta)
    if beta == 0.0:
        assert T6 == 2 ** 32
    elif math.isinf(beta):
        assert T6 == 0
    else:
        getcontext().prec = 60
        exact = (Decimal(-12) * Decimal(beta)).exp() * (Decimal(2) ** 32)
        ceil = int(exact.to_integral_value(rounding="ROUND_CEILING"))
        assert abs(exact - ceil) > Decimal("1e-4")      # no rounding tie at these beta
        assert T6 == ceil


@pytest.mark.parametrize("L,seed", [(2, 1), (4, 2), (6, 3)])
def test_local_field3_matches_roll_sum(oracle_lib, L, seed):
    s = _random(L, seed)
    assert np.array_equal(oracle_lib.local_field3(s).astype(np.int64), _roll_field(s))


def test_observables3(oracle_lib):
    for L, seed in ((2, 5), (4, 6), (8, 7)):
        s = _random(L, seed)
        si = s.astype(np.int64)
        E = -sum(int((si * np.roll(si, -1, axis=ax)).sum()) for ax in (0, 1, 2))
        assert oracle_lib.observables3(s) == (int(si.sum()), E)
    L, N = 6, 216
    assert oracle_lib.observables3(np.ones((L, L, L), dtype=np.int8)) == (N, -3 * N)
    neel = np.where(_parity(L) == 0, 1, -1).astype(np.int8)
    assert oracle_lib.observables3(neel) == (0, 3 * N)


def test_init3_is_the_row_contract(oracle_lib):
    L, seed = 4, 11
    s = oracle_lib.init3(L, seed)
    for z in range(L):
        for y in range(L):
            for x in range(L):
                assert s[z, y, x] == oracle_lib.init_site(seed, z * L + y, x)
    big = oracle_lib.init3(32, 12)
    assert abs(float((big == -1).mean()) - 0.5) < 5 * 0.5 / math.sqrt(big.size)


def test_beta_zero_flips_every_spin(oracle_lib):
    s0 = _random(6, 21)
    s = s0.copy()
    oracle_lib.sweep3(s, 0.0, 1, 9)
    assert np.array_equal(s, -s0)


def test_zero_temperature_from_neel(oracle_lib):
    L = 8
    s = np.where(_parity(L) == 0, 1, -1).astype(np.int8)   # white sites -1, all six neighbours +1
    oracle_lib.sweep3(s, math.inf, 1, 3)
    assert (s == 1).all()                                  # white flip; black then see s = 6


def test_half_sweep3_follows_the_uniform_contract(oracle_lib):
    L, beta, seed, t, q = 4, 0.2, 77, 5, 1
    s0 = _random(L, 31)
    s = s0.copy()
    oracle_lib.half_sweep3(s, beta, seed, t, q)
    T = oracle_lib.thresholds3(beta)
    nn = _roll_field(s0)
    for z in range(L):
        for y in range(L):
            for x in range(L):
                if (x + y + z) & 1 != q:
                    assert s[z, y, x] == s0[z, y, x]
                    continue
                sv = int(s0[z, y, x]) * int(nn[z, y, x])
                flip = sv <= 0 or oracle_lib.uniform(seed, z * L + y, x, t, q) < T[sv // 2 - 1]
                assert s[z, y, x] == (-s0[z, y, x] if flip else s0[z, y, x])


def _flip_fraction_test(oracle_lib, s0, beta, classes):
    """One white half-sweep; within each class (mask, s) every white site has local field s."""
    L = s0.shape[0]
    s = s0.copy()
    oracle_lib.half_sweep3(s, beta, 1234, 0, 1)
    white = _parity(L) == 1
    assert np.array_equal(s[~white], s0[~white])
    T = oracle_lib.thresholds3(beta)
    nn = _roll_field(s0)
    for mask, sval in classes:
        sel = mask & white
        assert np.all(s0[sel].astype(np.int64) * nn[sel] == sval)
        k = int((s[sel] != s0[sel]).sum())
        n = int(sel.sum())
        p = 1.0 if sval <= 0 else T[sval // 2 - 1] / 2 ** 32
        if p == 1.0:
            assert k == n
        else:
            assert abs(k - n * p) < 5 * math.sqrt(n * p * (1 - p)), (sval, k, n, p)


def test_flip_frequencies_for_every_local_field(oracle_lib):
    L, beta = 64, 0.15
    z = np.indices((L, L, L))[0]
    black = _parity(L) == 0
    # all +1: every white site has s = 6
    _flip_fraction_test(oracle_lib, np.ones((L, L, L), dtype=np.int8), beta, [(np.ones_like(black), 6)])
    # black -1 on planes z = 0 mod 4: white sites of odd planes have one anti-aligned neighbour
    # (s = 4), of planes 2 mod 4 none (s = 6), of planes 0 mod 4 four (s = -2)
    sB = np.where(black & (z % 4 == 0), -1, 1).astype(np.int8)
    _flip_fraction_test(oracle_lib, sB, beta, [(z % 2 == 1, 4), (z % 4 == 2, 6), (z % 4 == 0, -2)])
    # black -1 on even planes: white sites of odd planes have two anti-aligned neighbours (s = 2)
    sC = np.where(black & (z % 2 == 0), -1, 1).astype(np.int8)
    _flip_fraction_test(oracle_lib, sC, beta, [(z % 2 == 1, 2), (z % 2 == 0, -2)])


@pytest.mark.parametrize("beta", [0.1, 0.2, 0.35])
def test_l2_chain_matches_enumeration(oracle_lib, beta):
    L, N = 2, 8
    s = oracle_lib.init3(L, int(beta * 1000) + 5)
    oracle_lib.sweep3(s, beta, 1000, 77, 0)
    tr = oracle_lib.sweep3(s, beta, 200_000, 77, 1000, trace=True)
    m, e = tr[:, 0] / N, tr[:, 1] / N
    exact = X.boltzmann_moments3(L, beta)
    for series, key in ((e, "e"), (np.abs(m), "abs_m"), (m * m, "m2"), (m ** 4, "m4")):
        mean, err, _ = A.mean_err(series)
        assert abs(mean - exact[key]) < Z_MAX * err, (key, mean, exact[key], err)


def test_enumeration3_pins():
    # 2 x 2 x 2 torus: 3 bonds per site, 24 in all (two parallel bonds between each neighbour
    # pair); the two uniform states have E = -24, the two Neel states +24, and M sums to zero.
    E, M = X.enumerate_states3(2)
    assert E.min() == -24 and E.max() == 24
    assert int((E == -24).sum()) == 2 and int((E == 24).sum()) == 2
    assert int(M.sum()) == 0 and len(E) == 256


def test_crop3_matches_full_run(oracle_lib):
    L, n, seed, beta = 32, 2, 4, 0.25
    full = oracle_lib.init3(L, seed)
    oracle_lib.sweep3(full, beta, n, seed, 3)
    for (z0, y0, x0, d, h, w) in [(30, 1, 29, 4, 5, 6), (10, 20, 0, 3, 3, 3)]:
        blk = oracle_lib.crop3(L, seed, beta, n, 3, z0, y0, x0, d, h, w)
        zz = [(z0 + a) % L for a in range(d)]
        yy = [(y0 + a) % L for a in range(h)]
        xx = [(x0 + a) % L for a in range(w)]
        assert np.array_equal(blk, full[np.ix_(zz, yy, xx)])
