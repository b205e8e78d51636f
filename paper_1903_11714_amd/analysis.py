"""Statistics of Markov-chain time series and the exact 2D Ising results they are judged against.

* ``tau_int``: integrated autocorrelation time with Sokal's automatic window (the smallest W with
  W >= c tau(W)); ``mean_err`` turns it into the standard error sqrt(2 tau var / n).
* ``jackknife``: block jackknife of a function of series means, e.g. the Binder cumulant
  U4 = 1 - <m^4> / (3 <m^2>^2) of Sec. 4.1.
* ``onsager_energy`` (Onsager 1944) and ``yang_magnetisation`` (Yang 1952): the infinite-lattice
  energy per site and spontaneous magnetisation; T_c = 2 / ln(1 + sqrt 2) (Sec. 4.1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ellipk

T_C = 2.0 / math.log1p(math.sqrt(2.0))
BETA_C = 1.0 / T_C


def tau_int(x, c: float = 6.0) -> float:
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 4 or x.var() == 0.0:
        return 0.5
    d = x - x.mean()
    spec = np.fft.rfft(d, 2 * n)
    acf = np.fft.irfft(spec * np.conj(spec))[:n]
    acf /= acf[0]
    tau = 0.5
    for w in range(1, n):
        tau += acf[w]
        if w >= c * tau:
            break
    return max(tau, 0.5)


def mean_err(x):
    """(mean, autocorrelation-corrected standard error, tau_int)."""
    x = np.asarray(x, dtype=np.float64)
    tau = tau_int(x)
    err = math.sqrt(2.0 * tau * x.var(ddof=1) / x.size) if x.size > 1 else 0.0
    return float(x.mean()), err, tau


def jackknife(func, series, n_blocks: int = 50):
    """Block-jackknife estimate and error of func(mean(s1), mean(s2), ...)."""
    arrs = [np.asarray(s, dtype=np.float64) for s in series]
    b = arrs[0].size // n_blocks
    if b < 1:
        raise ValueError("series too short")
    sums = [a[: b * n_blocks].reshape(n_blocks, b).sum(axis=1) for a in arrs]
    tot = [s.sum() for s in sums]
    est = func(*[t / (b * n_blocks) for t in tot])
    loo = np.array([func(*[(t - s[k]) / (b * (n_blocks - 1)) for t, s in zip(tot, sums)])
                    for k in range(n_blocks)])
    err = math.sqrt((n_blocks - 1) / n_blocks * ((loo - loo.mean()) ** 2).sum())
    return float(est), err


def binder(m2: float, m4: float) -> float:
    return 1.0 - m4 / (3.0 * m2 * m2)


def z(a: float, ea: float, b: float, eb: float) -> float:
    d = math.sqrt(ea * ea + eb * eb)
    return (a - b) / d if d > 0 else 0.0


def onsager_energy(beta: float) -> float:
    k2b = 2.0 * beta
    factor = 2.0 * math.tanh(k2b) ** 2 - 1.0
    if abs(factor) < 1e-15:
        return -1.0 / math.tanh(k2b)
    kappa = 2.0 * math.sinh(k2b) / math.cosh(k2b) ** 2
    return -(1.0 / math.tanh(k2b)) * (1.0 + (2.0 / math.pi) * factor * float(ellipk(kappa * kappa)))


def yang_magnetisation(beta: float) -> float:
    return (1.0 - math.sinh(2.0 * beta) ** -4) ** 0.125 if beta > BETA_C else 0.0
