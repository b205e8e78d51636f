"""Pin the exact finite-lattice results (enumeration, Kaufman) against each other and against closed
forms.  These are what the oracle's Markov chain is later judged against (the infinite-lattice
closed forms are pinned in tests/test_analysis.py).
"""
import math

import pytest

from oracle import exact as X


def test_critical_point():
    # Sec. 4.1: T_c = 2 / ln(1 + sqrt 2)
    assert X.T_C == pytest.approx(2.0 / math.log(1 + math.sqrt(2)), rel=1e-15)
    assert X.T_C == pytest.approx(2.269185314213022, rel=1e-14)


@pytest.mark.parametrize("beta", [0.05, 0.2, 0.35, X.BETA_C, 0.47, 0.6, 1.0])
def test_enumeration_matches_kaufman(beta):
    # Two independent routes to ln Z of the 4 x 4 torus.
    assert X.boltzmann_moments(4, beta)["log_z"] == pytest.approx(X.kaufman_log_z(beta, 4, 4), rel=1e-12)


def test_enumeration_rectangular_kaufman():
    # Kaufman's formula for a 2 x 4 and 4 x 2 torus via brute force over 2^8 states.
    import itertools
    import numpy as np
    for m, n in ((2, 4), (4, 2)):
        for beta in (0.3, 0.7):
            Z = 0.0
            for bits in itertools.product((1, -1), repeat=m * n):
                s = np.array(bits).reshape(m, n)
                E = -(s * np.roll(s, -1, 1)).sum() - (s * np.roll(s, -1, 0)).sum()
                Z += math.exp(-beta * E)
            assert math.log(Z) == pytest.approx(X.kaufman_log_z(beta, m, n), rel=1e-12)


def test_density_of_states_combinatorics():
    g = X.density_of_states(4)
    assert sum(g.values()) == 2 ** 16
    assert all(E % 4 == 0 for E in g)
    assert all(g[E] == g.get(-E) for E in g)      # bipartite lattice: E -> -E symmetry
    assert g[-32] == 2                            # the two ground states
    assert g[-24] == 2 * 16                       # one flipped spin (4 broken bonds, +8)
    assert g[-20] == 2 * 32                       # a flipped nearest-neighbour pair (+12)
    assert -28 not in g                           # no excitation costs +4


def test_infinite_temperature_moments():
    mo = X.boltzmann_moments(4, 0.0)
    N = 16
    assert mo["e"] == pytest.approx(0.0, abs=1e-15)
    assert mo["m2"] == pytest.approx(1.0 / N)                     # <M^2> = N for iid spins
    assert mo["m4"] == pytest.approx((3 * N * N - 2 * N) / N ** 4)
    assert mo["U4"] == pytest.approx(2.0 / (3 * N))


def test_energy_derivative_of_log_z():
    # <E> = -d ln Z / d beta, from Kaufman by central differences.
    for beta in (0.3, X.BETA_C, 0.55):
        h = 1e-5
        dlz = (X.kaufman_log_z(beta + h, 4, 4) - X.kaufman_log_z(beta - h, 4, 4)) / (2 * h)
        assert X.boltzmann_moments(4, beta)["e"] * 16 == pytest.approx(-dlz, rel=1e-7)
