"""Error bars for Markov-chain time series (TEST INFRASTRUCTURE ONLY).

* ``tau_int``: integrated autocorrelation time with Sokal's automatic window (the smallest
  window W with W >= c * tau(W)).
* ``mean_and_error``: sample mean and its standard error sqrt(2 tau var / n).
* ``jackknife``: block-jackknife mean and error of a function of several series' means
  (used for the Binder cumulant U4 = 1 - <m^4> / (3 <m^2>^2), Sec. 4.1).
* ``z_score``: difference of two estimates in units of their combined standard error.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np


def autocorrelation(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    d = x - x.mean()
    f = np.fft.rfft(d, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    if acf[0] <= 0:
        return np.ones(1)
    return acf / acf[0]


def tau_int(x: np.ndarray, c: float = 6.0) -> float:
    rho = autocorrelation(x)
    if rho.size == 1:
        return 0.5
    tau = 0.5
    for W in range(1, rho.size):
        tau += rho[W]
        if W >= c * tau:
            return max(tau, 0.5)
    return max(tau, 0.5)


def mean_and_error(x: np.ndarray) -> tuple[float, float, float]:
    """(mean, standard error corrected for autocorrelation, tau_int)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    tau = tau_int(x)
    var = x.var(ddof=1) if n > 1 else 0.0
    return float(x.mean()), math.sqrt(2.0 * tau * var / n), tau


def jackknife(func: Callable[..., float], series: Sequence[np.ndarray], n_blocks: int = 32):
    """Block jackknife of func(mean(s1), mean(s2), ...); returns (estimate, error)."""
    arrs = [np.asarray(s, dtype=np.float64) for s in series]
    n = arrs[0].size
    b = n // n_blocks
    if b < 1:
        raise ValueError("series too short for the requested number of blocks")
    arrs = [a[: b * n_blocks].reshape(n_blocks, b) for a in arrs]
    sums = [a.sum(axis=1) for a in arrs]
    totals = [s.sum() for s in sums]
    full = func(*[t / (b * n_blocks) for t in totals])
    leave = np.array([
        func(*[(t - s[k]) / (b * (n_blocks - 1)) for t, s in zip(totals, sums)])
        for k in range(n_blocks)
    ])
    err = math.sqrt((n_blocks - 1) / n_blocks * ((leave - leave.mean()) ** 2).sum())
    return float(full), err


def binder(m2: float, m4: float) -> float:
    return 1.0 - m4 / (3.0 * m2 * m2)


def z_score(a: float, ea: float, b: float, eb: float) -> float:
    den = math.sqrt(ea * ea + eb * eb)
    return (a - b) / den if den > 0 else (0.0 if a == b else math.inf)
