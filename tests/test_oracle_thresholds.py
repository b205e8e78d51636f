"""Pin the integer acceptance thresholds.

Algorithm 1 (Sec. 3.2) flips a site when a uniform in [0, 1) is below the acceptance ratio
exp(-2 beta sigma nn) (beta restored in the exponent, as the Boltzmann weight of Sec. 3
requires).  With u = x / 2^32 for a 32-bit integer x, u < p holds exactly when
x < ceil(p 2^32), so the oracle stores T_s = ceil(2^32 exp(-2 beta s)) for s = 2, 4.
"""
import math
from decimal import Decimal, getcontext

import pytest

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))


def test_thresholds_at_critical_point_closed_form(oracle_lib):
    # exp(-2 beta_c) = sqrt 2 - 1, so p_2 = 3 - 2 sqrt 2 and p_4 = 17 - 12 sqrt 2 exactly.
    # ceil((a - sqrt(b)) 2^32) = a 2^32 - floor(sqrt(b 2^64)), with an exact integer sqrt.
    t2_exact = 3 * 2**32 - math.isqrt(8 * 2**64)
    t4_exact = 17 * 2**32 - math.isqrt(288 * 2**64)
    t2, t4 = oracle_lib.thresholds(BETA_C)
    # beta_c itself is a double; its rounding moves p by far less than one unit of 2^-32.
    assert (t2, t4) == (t2_exact, t4_exact)


def test_threshold_limits(oracle_lib):
    assert oracle_lib.thresholds(0.0) == (2**32, 2**32)        # every proposal accepted
    assert oracle_lib.thresholds(math.inf) == (0, 0)           # zero temperature: none
    assert oracle_lib.thresholds(1e6) == (0, 0)


@pytest.mark.parametrize("beta", [0.5, BETA_C, 0.4, 1 / 2.6, 0.1, 0.3, 1.0, 2.0, 5.0, 1e-9])
def test_threshold_brackets_probability(oracle_lib, beta):
    # (T - 1) / 2^32 < p <= T / 2^32 with p computed to 50 digits from the same double beta.
    getcontext().prec = 50
    b = Decimal(beta)
    for T, s in zip(oracle_lib.thresholds(beta), (2, 4)):
        p = (-2 * b * s).exp()
        scale = Decimal(2) ** 32
        assert Decimal(T - 1) / scale < p <= Decimal(T) / scale


def test_threshold_monotone(oracle_lib):
    prev = (2**32, 2**32)
    for k in range(1, 200):
        t2, t4 = oracle_lib.thresholds(k * 0.01)
        assert t4 <= t2 <= 2**32
        assert t2 <= prev[0] and t4 <= prev[1]
        prev = (t2, t4)
