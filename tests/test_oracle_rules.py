"""Pin the oracle's sweep against what the paper and the mathematics fix exactly.

Sec. 3      H = -sum_<ij> s_i s_j on a torus (J = 1, mu = 0).
Sec. 3.1    checkerboard: fixing one colour, every site of the other colour is updated
            independently; white sites first, then black.
Sec. 3.2    nn = sigma K + K sigma on 128 x 128 sub-lattices plus the neighbours taken from
            adjacent sub-lattices (Algorithm 1); the compact form on the four stride-2
            sub-lattices with the bidiagonal K-hat (Algorithm 2); flip where the uniform is
            below exp(-2 beta nn sigma); sigma -> sigma - 2 flips sigma.
"""
import math

import numpy as np
import pytest

from tests import inputs

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))


# ---------------------------------------------------------------- neighbour field (Sec. 3.2)

def _blocks(s, b):
    L = s.shape[0]
    m = L // b
    return s.reshape(m, b, m, b).transpose(0, 2, 1, 3)      # [m, n, b, b] grid of sub-lattices


def _unblocks(x):
    m, n, b, _ = x.shape
    return x.transpose(0, 2, 1, 3).reshape(m * b, n * b)


def _nn_algorithm1(s, b):
    """nn via K (tridiagonal, zero diagonal) per sub-lattice plus boundary compensation."""
    sig = _blocks(s.astype(np.int64), b)
    K = np.eye(b, k=1, dtype=np.int64) + np.eye(b, k=-1, dtype=np.int64)
    nn = sig @ K + K @ sig
    nn[:, :, 0, :] += np.roll(sig[:, :, -1, :], 1, axis=0)    # north: last row of block above
    nn[:, :, -1, :] += np.roll(sig[:, :, 0, :], -1, axis=0)   # south: first row of block below
    nn[:, :, :, 0] += np.roll(sig[:, :, :, -1], 1, axis=1)    # west: last column of left block
    nn[:, :, :, -1] += np.roll(sig[:, :, :, 0], -1, axis=1)   # east: first column of right block
    return _unblocks(nn)


def _nn_algorithm2(s, b):
    """nn of the four compact sub-lattices with the upper-bidiagonal K-hat (Alg. 2), with the
    boundary terms as the index algebra requires (the printed listing has slips in a few
    boundary lines: a wrong sub-lattice name and '=' for '+=')."""
    sig = _blocks(s.astype(np.int64), b)
    s00, s01 = sig[:, :, 0::2, 0::2], sig[:, :, 0::2, 1::2]
    s10, s11 = sig[:, :, 1::2, 0::2], sig[:, :, 1::2, 1::2]
    h = b // 2
    Kh = np.eye(h, dtype=np.int64) + np.eye(h, k=1, dtype=np.int64)
    KhT = Kh.T
    nn00 = s01 @ Kh + KhT @ s10
    nn00[:, :, 0, :] += np.roll(s10[:, :, -1, :], 1, axis=0)
    nn00[:, :, :, 0] += np.roll(s01[:, :, :, -1], 1, axis=1)
    nn11 = Kh @ s01 + s10 @ KhT
    nn11[:, :, -1, :] += np.roll(s01[:, :, 0, :], -1, axis=0)
    nn11[:, :, :, -1] += np.roll(s10[:, :, :, 0], -1, axis=1)
    nn01 = s00 @ KhT + KhT @ s11
    nn01[:, :, 0, :] += np.roll(s11[:, :, -1, :], 1, axis=0)
    nn01[:, :, :, -1] += np.roll(s00[:, :, :, 0], -1, axis=1)
    nn10 = Kh @ s00 + s11 @ Kh
    nn10[:, :, -1, :] += np.roll(s00[:, :, 0, :], -1, axis=0)
    nn10[:, :, :, 0] += np.roll(s11[:, :, :, -1], 1, axis=1)
    out = np.zeros_like(sig)
    out[:, :, 0::2, 0::2] = nn00
    out[:, :, 0::2, 1::2] = nn01
    out[:, :, 1::2, 0::2] = nn10
    out[:, :, 1::2, 1::2] = nn11
    return _unblocks(out)


@pytest.mark.parametrize("L,b", [(16, 4), (32, 8), (48, 16), (64, 64), (8, 2)])
def test_local_field_equals_matmul_formulations(oracle_lib, L, b):
    s = inputs.random_lattice(L, seed=L * 7 + b)
    nn = oracle_lib.local_field(s).astype(np.int64)
    assert np.array_equal(nn, _nn_algorithm1(s, b))
    assert np.array_equal(nn, _nn_algorithm2(s, b))


# ---------------------------------------------------------------- observables (Sec. 3, 4.1)

def test_observables_closed_forms(oracle_lib):
    L = 32
    assert oracle_lib.observables(inputs.all_up(L)) == (L * L, -2 * L * L)
    assert oracle_lib.observables(-inputs.all_up(L)) == (-L * L, -2 * L * L)
    assert oracle_lib.observables(inputs.neel(L)) == (0, 2 * L * L)
    # stripes of width w: every vertical bond aligned, horizontal bonds broken at 2 L/(2w) walls
    w = 4
    walls = L // w
    assert oracle_lib.observables(inputs.stripes(L, w)) == (0, -2 * L * L + 2 * walls * L)


def test_observables_match_bond_count(oracle_lib):
    # E = (#anti-aligned bonds) - (#aligned bonds) over the 2 L^2 bonds; M = #up - #down.
    s = inputs.random_lattice(40, seed=3)
    right = (s != np.roll(s, -1, axis=1)).sum()
    down = (s != np.roll(s, -1, axis=0)).sum()
    anti = int(right + down)
    E = anti - (2 * 40 * 40 - anti)
    M = int((s == 1).sum() - (s == -1).sum())
    assert oracle_lib.observables(s) == (M, E)


# ---------------------------------------------------------------- special temperatures

def test_infinite_temperature_flips_every_site(oracle_lib):
    # beta = 0: min{1, e^0} = 1, so every proposal is accepted; each sweep negates the lattice.
    s0 = inputs.random_lattice(32, seed=11)
    for n in (1, 2, 3, 7):
        s = s0.copy()
        oracle_lib.sweep(s, 0.0, n, seed=5)
        assert np.array_equal(s, s0 * (-1) ** n)


def test_neel_state_zero_temperature_pins_colour_order(oracle_lib):
    # White ((r+c) odd) = -1, black = +1.  The white half-sweep runs first: every white site
    # sees four +1 neighbours, s = -4 <= 0, and flips; the lattice is all +1.  Black sites then
    # see s = +4 and never flip at beta = inf.  (Black first would end at all -1.)
    L = 32
    s = inputs.neel(L, white=-1)
    tr = oracle_lib.sweep(s, math.inf, 1, seed=1, trace=True)
    assert np.array_equal(s, inputs.all_up(L))
    assert tuple(tr[0]) == (L * L, -2 * L * L)


def test_neel_state_black_flip_fraction(oracle_lib):
    # After the white half-sweep makes the lattice all +1, each black site flips with
    # probability exactly T_4 / 2^32 (s = 4, independent draws).  Binomial 5-sigma check.
    L, beta = 128, 0.15
    s = inputs.neel(L, white=-1)
    oracle_lib.sweep(s, beta, 1, seed=21)
    black = ((np.indices((L, L)).sum(axis=0)) % 2 == 0)
    flipped = int((s[black] == -1).sum())
    n = int(black.sum())
    p = oracle_lib.thresholds(beta)[1] / 2**32
    assert abs(flipped - n * p) < 5 * math.sqrt(n * p * (1 - p))
    assert (s[~black] == 1).all()


def test_zero_temperature_isolated_spin_flips_back(oracle_lib):
    # A lone -1 in a +1 sea has s = sigma nn = -4 (the flip lowers the energy by 8) and flips
    # in its colour's half-sweep; its +1 neighbours have s = +2 and stay at beta = inf.
    L = 32
    for (r, c) in ((10, 13), (10, 14), (0, 0), (31, 30)):
        s = inputs.all_up(L)
        s[r, c] = -1
        oracle_lib.sweep(s, math.inf, 1, seed=2)
        assert np.array_equal(s, inputs.all_up(L))


def test_zero_temperature_flips_majority_minority(oracle_lib):
    # s = 0 (two aligned, two anti-aligned neighbours) flips with probability 1 (Sec. 3.2:
    # min{1, exp(0)} = 1), while s = +2 never flips at T = 0.
    L = 32
    s = inputs.all_up(L)
    # a straight domain wall: rows 0..15 = -1, rows 16..31 = +1; sites on the wall have
    # s = 4 - 2a with a = 1, so s = 2 > 0: stable at T = 0.
    s[:16, :] = -1
    s0 = s.copy()
    oracle_lib.sweep(s, math.inf, 2, seed=3)
    assert np.array_equal(s, s0)
    # a corner of a -1 square: site (0, 0) of a 4x4 -1 block in a +1 sea has two -1 and two
    # +1 neighbours -> s = 0 -> flips in its half-sweep.
    s = inputs.all_up(L)
    s[8:12, 8:12] = -1
    oracle_lib.half_sweep(s, math.inf, seed=3, t=0, q=0)       # (8, 8) is black
    assert s[8, 8] == 1 and s[11, 11] == 1                      # both black corners flipped
    assert s[8, 11] == -1 and s[11, 8] == -1                    # white corners untouched


# ---------------------------------------------------------------- contract properties

def test_sweep_chunks_compose(oracle_lib):
    # The random numbers depend only on (site, sweep index, colour): running n1 sweeps and then
    # n2 more from offset n1 equals running n1 + n2 sweeps.
    s_a = oracle_lib.init(64, seed=9)
    s_b = s_a.copy()
    oracle_lib.sweep(s_a, BETA_C, 7, seed=9, offset=3)
    oracle_lib.sweep(s_b, BETA_C, 4, seed=9, offset=3)
    oracle_lib.sweep(s_b, BETA_C, 3, seed=9, offset=7)
    assert np.array_equal(s_a, s_b)


def test_trace_matches_recomputed_observables(oracle_lib):
    s = oracle_lib.init(48, seed=4)
    ref = s.copy()
    tr = oracle_lib.sweep(s, 0.42, 20, seed=4, trace=True)
    for i in range(20):
        oracle_lib.sweep(ref, 0.42, 1, seed=4, offset=i)
        assert tuple(tr[i]) == oracle_lib.observables(ref)
    assert ((s == 1) | (s == -1)).all()
    assert np.all(tr[:, 1] % 4 == 0) and np.all(tr[:, 0] % 2 == 0)
    assert np.all(np.abs(tr[:, 1]) <= 2 * 48 * 48)


def test_half_sweep_only_touches_its_colour(oracle_lib):
    s = oracle_lib.init(64, seed=8)
    s0 = s.copy()
    oracle_lib.half_sweep(s, 0.3, seed=8, t=5, q=1)
    odd = (np.indices(s.shape).sum(axis=0) % 2 == 1)
    assert np.array_equal(s[~odd], s0[~odd])
    assert (s[odd] != s0[odd]).any()


@pytest.mark.parametrize("L,n,r0,c0,h,w", [
    (64, 3, 10, 20, 8, 12),
    (64, 2, 60, 62, 9, 5),      # crosses both seams
    (96, 5, 0, 0, 16, 16),
    (64, 10, 5, 5, 6, 6),       # window would cover the torus: falls back to the full lattice
])
def test_light_cone_crop_equals_full_lattice(oracle_lib, L, n, r0, c0, h, w):
    beta, seed, offset = BETA_C, 17, 11
    full = oracle_lib.init(L, seed)
    oracle_lib.sweep(full, beta, n, seed, offset)
    rows = [(r0 + a) % L for a in range(h)]
    cols = [(c0 + b) % L for b in range(w)]
    expect = full[np.ix_(rows, cols)]
    got = oracle_lib.crop(L, seed, beta, n, offset, r0, c0, h, w)
    assert np.array_equal(got, expect)


def test_init_is_balanced_and_seeded(oracle_lib):
    a = oracle_lib.init(128, seed=1)
    b = oracle_lib.init(128, seed=2)
    assert ((a == 1) | (a == -1)).all()
    assert abs(int(a.sum())) < 5 * 128                    # 5 sigma of a fair +-1 sum
    assert (a != b).mean() > 0.45
    assert oracle_lib.init_site(1, 5, 77) == a[5, 77]


def test_init_has_no_repeated_rows_or_columns(oracle_lib):
    # The hot start draws every site's bit from its own (row, 128-column chunk, word, bit) position of
    # the init stream; a mapping that reused a counter or a word would repeat rows or columns.  Among
    # 512 random rows (or columns) of 512 spins, two equal ones have probability ~2^-494.
    a = oracle_lib.init(512, seed=9)
    assert len({row.tobytes() for row in a}) == 512
    assert len({col.tobytes() for col in a.T}) == 512
    # neighbouring columns across a word (32) and chunk (128) boundary are uncorrelated
    for d in (1, 32, 128):
        corr = float((a[:, :-d].astype(np.int64) * a[:, d:]).mean())
        assert abs(corr) < 5 / math.sqrt(a[:, d:].size), d


def test_init_site_uses_the_init_stream(oracle_lib):
    # sigma0(r, c) = -1 iff bit c & 31 of word (c >> 5) & 3 of Philox(key, (c >> 7, r, 0, 2^31)); the
    # generator itself is pinned against rocRAND (test_oracle_philox.py)
    seed = 0x1234_5678_9ABC_DEF0
    rng = np.random.default_rng(5)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for _ in range(200):
        r, c = int(rng.integers(0, 1 << 20)), int(rng.integers(0, 1 << 20))
        blk = oracle_lib.philox4x32_10([c >> 7, r, 0, 0x80000000], key)
        bit = (int(blk[(c >> 5) & 3]) >> (c & 31)) & 1
        assert oracle_lib.init_site(seed, r, c) == (-1 if bit else 1)
