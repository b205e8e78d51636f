"""Pins of the statistics and closed forms in ``paper_1903_11714_amd/analysis.py``.

Every error bar of the oracle's stationarity tests and of the two form studies comes from these
routines, so each one is checked against something other than itself:

* tau_int against AR(1) series, whose integrated autocorrelation time is (1 + rho) / (2 (1 - rho)),
  and iid data (tau = 1/2);
* the error of the mean against the exact variance of the mean of a finite AR(1) series;
* the jackknife against its algebraic identities (a plain mean gives the naive standard error of the
  block means) and, for the Binder cumulant, against the delta method on Gaussian data, where the
  moments E m^2k = (2k - 1)!! fix the answer;
* the paired forms against chains whose difference is known in law;
* Onsager's energy against Kaufman's exact finite-torus partition function (an independent route:
  -d ln Z / d beta on a 128 x 128 torus, whose finite-size correction is exponentially small away
  from T_c) and its value -sqrt 2 at T_c;
* Yang's magnetisation against the low-temperature series 1 - 2x^4 - 8x^6 - 34x^8 (x = e^{-2 beta}),
  whose leading term is one flipped spin (weight x^4, magnetisation change 2 per site);
* the U4 crossing estimator against synthetic curves that cross at a known temperature.
"""
import math

import numpy as np
import pytest

from oracle import exact as X
from paper_1903_11714_amd import analysis as A


def ar1_fast(rng, rho, n):
    """One long AR(1) series via a linear filter (same law as ``ar1``)."""
    from scipy.signal import lfilter
    eps = rng.standard_normal(n)
    eps[0] /= math.sqrt(1 - rho * rho)
    return lfilter([1.0], [1.0, -rho], eps)


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_tau_int_of_ar1(rho):
    rng = np.random.default_rng(11)
    exact = (1 + rho) / (2 * (1 - rho))
    taus = [A.tau_int(ar1_fast(rng, rho, 1 << 18)) for _ in range(4)]
    # relative statistical error of one estimate ~ sqrt(2 (2W + 1) / n) <= 3% here
    assert np.mean(taus) == pytest.approx(exact, rel=0.05), (taus, exact)


def test_tau_int_of_iid_data_is_one_half():
    rng = np.random.default_rng(12)
    assert A.tau_int(rng.standard_normal(1 << 16)) == pytest.approx(0.5, abs=0.03)
    assert A.tau_int(np.ones(100)) == 0.5          # no fluctuation at all


def test_mean_error_matches_exact_variance_of_ar1_mean():
    # Var(mean) of n stationary AR(1) values: gamma0 / n [1 + 2 sum_t (1 - t / n) rho^t].
    rho, n, reps = 0.8, 8192, 200
    rng = np.random.default_rng(13)
    t = np.arange(1, n)
    gamma0 = 1.0 / (1 - rho * rho)
    var_mean = gamma0 / n * (1 + 2 * np.sum((1 - t / n) * rho ** t))
    errs = [A.mean_err(ar1_fast(rng, rho, n))[1] for _ in range(reps)]
    assert math.sqrt(np.mean(np.square(errs))) == pytest.approx(math.sqrt(var_mean), rel=0.06)


def test_jackknife_of_a_mean_is_the_standard_error_of_the_block_means():
    rng = np.random.default_rng(14)
    x = rng.standard_normal(6000) * 3 + 1
    for nb in (6000, 100, 20):
        est, err = A.jackknife(lambda a: a, [x], n_blocks=nb)
        blocks = x.reshape(nb, -1).mean(axis=1)
        assert est == pytest.approx(x.mean(), rel=1e-12)
        assert err == pytest.approx(blocks.std(ddof=1) / math.sqrt(nb), rel=1e-10)
    # block size 1: the naive standard error of the series
    assert A.jackknife(lambda a: a, [x], n_blocks=x.size)[1] == pytest.approx(x.std(ddof=1) / math.sqrt(x.size),
                                                                             rel=1e-10)


def test_jackknife_of_binder_cumulant_matches_delta_method():
    # m ~ N(0, 1): E m^2 = 1, E m^4 = 3, E m^6 = 15, E m^8 = 105.  For U4 = f(a, b) = 1 - b / (3 a^2) at
    # (a, b) = (1, 3): grad f = (2 b / (3 a^3), -1 / (3 a^2)) = (2, -1/3), Cov(m^2, m^4) =
    # [[2, 12], [12, 96]], so Var(U4) = (8 - 16 + 96 / 9) / n = (8 / 3) / n and U4 itself is 0.
    n = 1_000_000
    rng = np.random.default_rng(15)
    m = rng.standard_normal(n)
    u4, err = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=1000)
    delta = math.sqrt(8.0 / 3.0 / n)
    assert err == pytest.approx(delta, rel=0.1), (err, delta)
    assert abs(u4) < 5 * delta


def test_binder_limits():
    assert A.binder(1.0, 1.0) == pytest.approx(2.0 / 3.0)      # m = +-1: ordered
    assert A.binder(1.0, 3.0) == pytest.approx(0.0)            # Gaussian m: disordered


def test_paired_error_uses_the_difference_series():
    # y = x + c + eta with eta iid N(0, s^2): the difference has mean c and error s / sqrt(n), however
    # large and however autocorrelated x is; adding the two chains' errors in quadrature would be ~25x
    # larger here.
    rng = np.random.default_rng(16)
    n, c, s = 1 << 16, 0.01, 0.05
    x = ar1_fast(rng, 0.95, n)
    y = x + c + s * rng.standard_normal(n)
    d, err, tau = A.paired_mean_err(y, x)
    assert d == pytest.approx(c, abs=5 * s / math.sqrt(n))
    assert err == pytest.approx(s / math.sqrt(n), rel=0.05)
    assert tau == pytest.approx(0.5, abs=0.05)
    quad = math.hypot(A.mean_err(x)[1], A.mean_err(y)[1])
    assert quad > 10 * err


def test_paired_jackknife_keeps_the_correlation():
    rng = np.random.default_rng(17)
    m = rng.standard_normal(200_000)
    mm = m * (1 + 1e-3 * rng.standard_normal(m.size))           # nearly the same chain
    d, err = A.paired_jackknife(A.binder, [mm * mm, mm ** 4], [m * m, m ** 4], n_blocks=100)
    _, single = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=100)
    assert err < 0.05 * single and abs(d) < 5 * err


def test_seed_mean_error():
    v = np.array([1.0, 2.0, 4.0, 7.0])
    mean, err = A.seed_mean_err(v)
    assert mean == 3.5 and err == pytest.approx(math.sqrt(((v - 3.5) ** 2).sum() / 3 / 4))


def test_critical_temperature():
    # Sec. 4.1: T_c = 2 / ln(1 + sqrt 2); sinh 2 beta_c = 1
    assert A.T_C == pytest.approx(2.269185314213022, rel=1e-14)
    assert math.sinh(2 * A.BETA_C) == pytest.approx(1.0, rel=1e-14)
    assert A.BETA_C == pytest.approx(X.BETA_C, rel=1e-15)


@pytest.mark.parametrize("beta", [0.3, 0.4, 0.5, 0.6])
def test_onsager_energy_matches_kaufman_on_a_large_torus(beta):
    L, h = 128, 1e-5
    dlz = (X.kaufman_log_z(beta + h, L, L) - X.kaufman_log_z(beta - h, L, L)) / (2 * h)
    assert A.onsager_energy(beta) == pytest.approx(-dlz / (L * L), abs=1e-7)


def test_onsager_energy_special_values():
    assert A.onsager_energy(A.BETA_C) == pytest.approx(-math.sqrt(2), rel=1e-14)
    assert A.onsager_energy(A.BETA_C * (1 + 1e-7)) == pytest.approx(-math.sqrt(2), abs=1e-4)  # continuous
    assert A.onsager_energy(20.0) == pytest.approx(-2.0, abs=1e-12)      # ground state
    assert A.onsager_energy(1e-4) == pytest.approx(-2 * math.tanh(1e-4), rel=1e-3)  # high T: 2 bonds x tanh K


@pytest.mark.parametrize("T", [0.5, 0.7, 0.9])
def test_yang_magnetisation_matches_low_temperature_series(T):
    x = math.exp(-2.0 / T)
    series = 1 - 2 * x ** 4 - 8 * x ** 6 - 34 * x ** 8
    assert A.yang_magnetisation(1.0 / T) == pytest.approx(series, abs=200 * x ** 10)


def test_yang_magnetisation_limits():
    assert A.yang_magnetisation(A.BETA_C * 0.999) == 0.0
    assert A.yang_magnetisation(10.0) == pytest.approx(1.0, abs=1e-12)
    assert 0 < A.yang_magnetisation(A.BETA_C * 1.001) < 0.6   # rises as (T_c - T)^(1/8)


def _synthetic_m(rng, L, T, n, Tc, c):
    """iid m with U4 = 2 mu^4 / (3 (mu^2 + 1)^2) for m ~ N(+-mu, 1): mu = exp(c (Tc - T) L) equals 1 at
    T = Tc for every L, so the U4 curves of all sizes cross exactly at Tc."""
    mu = math.exp(c * (Tc - T) * L)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return sign * mu + rng.standard_normal(n)


def test_u4_crossing_estimate_and_its_jackknife_error():
    # A resolved crossing (one rising sign change of U4_8 - U4_16 on the grid): the estimates scatter
    # around Tc, and the jackknife error matches that scatter (24 repeats: the scatter itself is known
    # to about 15%; the ratio estimator's jackknife runs slightly high, never low).
    Tc, c, n = 2.275, 1.0, 50000
    temps = np.linspace(2.17, 2.37, 11)
    Ls = (8, 16)
    rng = np.random.default_rng(18)
    found, errs = [], []
    for _ in range(24):
        series = {L: [_synthetic_m(rng, L, T, n, Tc, c) for T in temps] for L in Ls}
        (res,) = A.u4_crossings(Ls, temps, series, n_blocks=40)
        assert res["pair"] == [8, 16] and res["bracket"] == pytest.approx([2.27, 2.29])
        found.append(res["T_cross"])
        errs.append(res["err"])
    found = np.array(found)
    # linear interpolation of the convex curves on this grid biases the estimate by ~1e-3
    assert abs(found.mean() - Tc) < 4 * found.std(ddof=1) / math.sqrt(found.size) + 2e-3
    ratio = np.sqrt(np.mean(np.square(errs))) / found.std(ddof=1)
    assert 0.7 < ratio < 1.5, ratio


def test_quadratic_crossing_is_exact_for_a_quadratic_difference():
    # d(T) = (T - 2.27)(T + 1) on a 0.012 grid: the quadratic through four points is d itself, while the
    # chord between the bracket's end points misses the root by the curvature term
    temps = np.round(np.arange(2.2, 2.35, 0.012), 6)
    d = (temps - 2.27) * (temps + 1.0)
    k = int(np.searchsorted(temps, 2.27)) - 1
    assert A._crossing_quad(temps, d, k) == pytest.approx(2.27, abs=1e-12)
    lin = A._crossing_in(temps, d, k)
    assert abs(lin - 2.27) > 1e-7
    d2 = (temps - 2.27) * (temps - 1.8) * 40.0          # stronger curvature, the same root
    assert A._crossing_quad(temps, d2, k) == pytest.approx(2.27, abs=1e-12)
    assert abs(A._crossing_in(temps, d2, k) - 2.27) > abs(lin - 2.27)


def test_crossing_reports_interpolation_error_and_combined_z():
    Tc, c, n = 2.275, 1.0, 20000
    temps = np.linspace(2.17, 2.37, 11)
    rng = np.random.default_rng(5)
    series = {L: [_synthetic_m(rng, L, T, n, Tc, c) for T in temps] for L in (8, 16)}
    (res,) = A.u4_crossings((8, 16), temps, series, n_blocks=20)
    assert res["syst"] == pytest.approx(abs(res["T_cross_quad"] - res["T_cross"]))
    assert abs(res["z_total"]) <= abs(res["z_vs_Tc"]) + 1e-12
    assert res["z_total"] == pytest.approx((res["T_cross"] - A.T_C) / math.hypot(res["err"], res["syst"]))
