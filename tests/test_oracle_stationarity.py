"""The oracle's chain samples the Boltzmann distribution (Sec. 3.1 eq. 1 and the appendix's
Metropolis-within-Gibbs stationarity proof).

* L = 4: long chains against the exact enumeration (2^16 states) at three temperatures.
* L = 64: the energy per site against Onsager at T = 2.5 and the magnetisation against Yang
  at T = 2.0 (finite-size corrections there are far below the statistical error).

Error bars are corrected for autocorrelation (Sokal windowing; the statistics routines are pinned
in tests/test_analysis.py); the bar is 4.5 sigma.
"""
import math

import numpy as np
import pytest

from oracle import exact as X
from paper_1903_11714_amd import analysis as A

Z_MAX = 4.5


def _run(oracle_lib, L, beta, n_burn, n_meas, seed, cold=False):
    s = np.ones((L, L), dtype=np.int8) if cold else oracle_lib.init(L, seed)
    oracle_lib.sweep(s, beta, n_burn, seed, 0)
    tr = oracle_lib.sweep(s, beta, n_meas, seed, n_burn, trace=True)
    N = L * L
    return tr[:, 0].astype(np.float64) / N, tr[:, 1].astype(np.float64) / N


@pytest.mark.parametrize("beta", [0.3, X.BETA_C, 0.5])
def test_l4_chain_matches_enumeration(oracle_lib, beta):
    m, e = _run(oracle_lib, 4, beta, 1000, 200_000, seed=int(beta * 1000) + 7)
    exact = X.boltzmann_moments(4, beta)
    for series, key in ((e, "e"), (np.abs(m), "abs_m"), (m * m, "m2"), (m ** 4, "m4")):
        mean, err, _ = A.mean_err(series)
        z = (mean - exact[key]) / err
        assert abs(z) < Z_MAX, (key, mean, exact[key], err, z)
    u4, u4_err = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=50)
    assert abs(u4 - exact["U4"]) < Z_MAX * u4_err


def test_l64_energy_matches_onsager_above_tc(oracle_lib):
    beta = 0.4                                      # T = 2.5
    _, e = _run(oracle_lib, 64, beta, 300, 4000, seed=101)
    mean, err, _ = A.mean_err(e)
    assert abs(mean - A.onsager_energy(beta)) < Z_MAX * err, (mean, A.onsager_energy(beta), err)
    assert err < 3e-3


def test_l64_magnetisation_matches_yang_below_tc(oracle_lib):
    beta = 0.5                                      # T = 2.0, cold start (ordered phase)
    m, e = _run(oracle_lib, 64, beta, 300, 4000, seed=202, cold=True)
    mean, err, _ = A.mean_err(np.abs(m))
    assert abs(mean - A.yang_magnetisation(beta)) < Z_MAX * err + 2e-4, (mean, err)
    emean, eerr, _ = A.mean_err(e)
    assert abs(emean - A.onsager_energy(beta)) < Z_MAX * eerr


def test_wrong_temperature_would_be_detected(oracle_lib):
    # Sensitivity check: a chain at 0.9 beta is many sigma away from Onsager at beta.
    beta = 0.4
    _, e = _run(oracle_lib, 64, 0.9 * beta, 300, 2000, seed=303)
    mean, err, _ = A.mean_err(e)
    assert abs(mean - A.onsager_energy(beta)) > 10 * err
