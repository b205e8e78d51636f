"""Statistics of Markov-chain time series, and the exact 2D Ising results the chains are judged by.

This is the one copy of these routines.  The studies of the two forms (``studies.py``) use it for
their error bars, and the tests that pin the CPU oracle's chains to exact results use it too; it is
itself pinned by ``tests/test_analysis.py`` (AR(1) series of known autocorrelation time, iid data,
algebraic identities of the jackknife, the delta method, Kaufman's finite torus and the
low-temperature series of the magnetisation).

* ``tau_int``: integrated autocorrelation time tau = 1/2 + sum_t rho(t), summed up to Sokal's
  automatic window (the smallest W with W >= c tau(W)); ``mean_err`` turns it into the standard
  error of the mean, sqrt(2 tau var / n).
* ``jackknife``: block jackknife of a function of series means, e.g. the Binder cumulant
  U4 = 1 - <m^4> / (3 <m^2>^2) of Sec. 4.1.
* ``paired_mean_err`` / ``paired_jackknife``: the same for the DIFFERENCE of two chains that share
  their random numbers (and are therefore correlated): the error comes from the difference series
  itself, not from the two errors added in quadrature.
* ``seed_mean_err``: mean and standard error over independent chains (one number per seed).
* ``onsager_energy`` (Onsager 1944) and ``yang_magnetisation`` (Yang 1952): the infinite-lattice
  energy per site and spontaneous magnetisation; T_c = 2 / ln(1 + sqrt 2) (Sec. 4.1).
* ``u4_crossings``: the temperature where the U4(T) curves of two lattice sizes cross (Sec. 4.1,
  the Binder-cumulant curves for several L), with a jackknife error over synchronised blocks of
  every replica's series.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np
from scipy.special import ellipk

T_C = 2.0 / math.log1p(math.sqrt(2.0))
BETA_C = 1.0 / T_C


# ---- autocorrelation ---------------------------------------------------------------------------

def autocorrelation(x) -> np.ndarray:
    """Normalised autocorrelation rho(t), t = 0 .. n - 1 (FFT over a zero-padded copy)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    d = x - x.mean()
    spec = np.fft.rfft(d, 2 * n)
    acf = np.fft.irfft(spec * np.conj(spec))[:n]
    if not acf[0] > 0:
        return np.ones(1)
    return acf / acf[0]


def tau_int(x, c: float = 6.0) -> float:
    """Integrated autocorrelation time with Sokal's automatic window (W >= c tau(W))."""
    x = np.asarray(x, dtype=np.float64)
    if x.size < 4:
        return 0.5
    rho = autocorrelation(x)
    if rho.size == 1:
        return 0.5
    tau = 0.5
    for w in range(1, rho.size):
        tau += rho[w]
        if w >= c * tau:
            break
    return max(tau, 0.5)


def mean_err(x):
    """(mean, standard error corrected for autocorrelation, tau_int)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    tau = tau_int(x)
    err = math.sqrt(2.0 * tau * x.var(ddof=1) / n) if n > 1 else 0.0
    return float(x.mean()), err, tau


# ---- jackknife ---------------------------------------------------------------------------------

def _block_sums(series: Sequence[np.ndarray], n_blocks: int):
    arrs = [np.asarray(s, dtype=np.float64) for s in series]
    b = arrs[0].size // n_blocks
    if b < 1:
        raise ValueError("series too short for the requested number of blocks")
    sums = [a[: b * n_blocks].reshape(n_blocks, b).sum(axis=1) for a in arrs]
    return sums, b


def jackknife_samples(func: Callable[..., float], series: Sequence[np.ndarray], n_blocks: int = 50):
    """(full estimate, leave-one-block-out estimates) of func(mean(s1), mean(s2), ...)."""
    sums, b = _block_sums(series, n_blocks)
    tot = [s.sum() for s in sums]
    full = func(*[t / (b * n_blocks) for t in tot])
    loo = np.array([func(*[(t - s[k]) / (b * (n_blocks - 1)) for t, s in zip(tot, sums)])
                    for k in range(n_blocks)])
    return float(full), loo


def jackknife_error(loo: np.ndarray) -> float:
    loo = np.asarray(loo, dtype=np.float64)
    nb = loo.size
    return math.sqrt((nb - 1) / nb * ((loo - loo.mean()) ** 2).sum())


def jackknife(func: Callable[..., float], series: Sequence[np.ndarray], n_blocks: int = 50):
    """Block-jackknife estimate and error of func(mean(s1), mean(s2), ...)."""
    full, loo = jackknife_samples(func, series, n_blocks)
    return full, jackknife_error(loo)


def binder(m2: float, m4: float) -> float:
    return 1.0 - m4 / (3.0 * m2 * m2)


def z(a: float, ea: float, b: float, eb: float) -> float:
    """(a - b) in units of the two errors added in quadrature (independent estimates only)."""
    d = math.sqrt(ea * ea + eb * eb)
    return (a - b) / d if d > 0 else 0.0


# ---- two chains that share their random numbers --------------------------------------------------

def paired_mean_err(x, y):
    """Mean of x - y over the time series, its autocorrelation-corrected error and tau_int of the
    difference.  Valid for correlated chains (same seed and random numbers): the error is that of
    the difference series, so the positive correlation is not counted twice."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return mean_err(d)


def paired_jackknife(func: Callable[..., float], xs: Sequence[np.ndarray], ys: Sequence[np.ndarray],
                     n_blocks: int = 50):
    """Jackknife of func(means of xs) - func(means of ys) with the same time blocks removed from both
    chains, so that their correlation is kept.  Returns (difference, error)."""
    fx, lx = jackknife_samples(func, xs, n_blocks)
    fy, ly = jackknife_samples(func, ys, n_blocks)
    return fx - fy, jackknife_error(lx - ly)


def seed_mean_err(values):
    """Mean and standard error over independent chains (one value per seed, ddof = 1)."""
    v = np.asarray(values, dtype=np.float64)
    if v.size < 2:
        return float(v.mean()), float("nan")
    return float(v.mean()), float(v.std(ddof=1) / math.sqrt(v.size))


# ---- exact infinite-lattice results --------------------------------------------------------------

def onsager_energy(beta: float) -> float:
    """Energy per site of the infinite square lattice (J = 1):
    -coth 2K [1 + (2 / pi)(2 tanh^2 2K - 1) K(k)], k = 2 sinh 2K / cosh^2 2K, K = beta
    (scipy's ellipk takes the parameter k^2)."""
    k2b = 2.0 * beta
    factor = 2.0 * math.tanh(k2b) ** 2 - 1.0
    if abs(factor) < 1e-15:  # at T_c the logarithmic divergence of K(k) is multiplied by zero
        return -1.0 / math.tanh(k2b)
    kappa = 2.0 * math.sinh(k2b) / math.cosh(k2b) ** 2
    return -(1.0 / math.tanh(k2b)) * (1.0 + (2.0 / math.pi) * factor * float(ellipk(kappa * kappa)))


def yang_magnetisation(beta: float) -> float:
    """Spontaneous magnetisation (1 - sinh^-4 2K)^(1/8) below T_c, 0 above."""
    return (1.0 - math.sinh(2.0 * beta) ** -4) ** 0.125 if beta > BETA_C else 0.0


# ---- Binder-cumulant crossings ------------------------------------------------------------------

def _crossing_in(temps, d, k):
    """Linear interpolation of the zero of d between temps[k] and temps[k + 1]."""
    slope = (d[k + 1] - d[k]) / (temps[k + 1] - temps[k])
    return float(temps[k] - d[k] / slope) if slope != 0 else float("nan")


def _crossing_quad(temps, d, k):
    """Zero of the least-squares quadratic through d at the four grid points around the bracket
    [temps[k], temps[k + 1]] (three at the ends of the grid), the one nearest the bracket."""
    lo, hi = max(0, k - 1), min(len(temps), k + 3)
    if hi - lo < 3:
        return _crossing_in(temps, d, k)
    x = np.asarray(temps[lo:hi], dtype=np.float64) - temps[k]
    c2, c1, c0 = np.polyfit(x, np.asarray(d[lo:hi], dtype=np.float64), 2)
    roots = np.roots([c2, c1, c0]) if c2 != 0 else np.array([-c0 / c1])
    roots = roots[np.isreal(roots)].real
    if roots.size == 0:
        return _crossing_in(temps, d, k)
    mid = 0.5 * (temps[k + 1] - temps[k])
    return float(temps[k] + roots[np.argmin(np.abs(roots - mid))])


def crossing_blocks(m_series_pair, n: int, max_blocks: int = 50, min_blocks: int = 8) -> int:
    """Jackknife blocks for a crossing: each block spans at least four tau_int of the slowest replica
    of the two sizes (tau_int of m^2 and |m|), between min_blocks and max_blocks blocks."""
    tau = max(max(tau_int(np.asarray(m, dtype=np.float64) ** 2), tau_int(np.abs(np.asarray(m, dtype=np.float64))))
              for m in m_series_pair)
    return int(max(min_blocks, min(max_blocks, n // max(1, int(math.ceil(4 * tau))))))


def u4_crossings(Ls, temps, m_series, n_blocks: int = 50) -> list:
    """Crossing temperatures of the U4(T) curves of neighbouring sizes a < b.

    m_series[L][i] is the magnetisation-per-site series of the replica (L, temps[i]).  Above T_c
    the smaller lattice has the larger U4 and below T_c the smaller one, so the crossing is a
    rising sign change of D(T) = U4_a(T) - U4_b(T).  Where the curves sit on a plateau (near 2/3
    below T_c, near 0 above) D is noise and can change sign by chance, so the bracket taken is the
    rising sign change whose two end points are largest in units of their errors.  The crossing is
    the linear interpolation of D's zero in that bracket.

    Interpolation: the zero of a quadratic through the four grid points around the bracket gives a
    second estimate; their difference is reported as the interpolation error (syst), which the
    jackknife does not see, and z_total divides by both errors in quadrature.

    Error: a jackknife over n_blocks synchronised time blocks.  Leaving block k out of EVERY
    replica's series (the replicas are independent chains, so any pairing of their blocks is a
    valid resampling) gives U4 curves, hence a crossing T_k in the same bracket; the error is
    sqrt((n - 1) / n sum_k (T_k - mean T_k)^2).  n_blocks may be a number, or a function of
    (list of the two sizes' series at the bracket's two temperatures, series length) that picks it
    per pair (crossing_blocks: blocks of at least four tau_int).
    """
    temps = np.asarray(temps, dtype=np.float64)

    def curves(L, nb):
        full, loo = [], []
        for m in m_series[L]:
            m = np.asarray(m, dtype=np.float64)
            f, lo = jackknife_samples(binder, [m * m, m ** 4], nb)
            full.append(f)
            loo.append(lo)
        return np.array(full), np.array(loo)  # (n_T,), (n_T, nb)

    def bracket(d, de):
        best = None
        for k in range(len(temps) - 1):
            if d[k] <= 0 < d[k + 1]:
                sig = (abs(d[k]) + abs(d[k + 1])) / max(de[k] + de[k + 1], 1e-300)
                if best is None or sig > best[0]:
                    best = (sig, k)
        return best

    out = []
    for a, b in zip(Ls[:-1], Ls[1:]):
        nb = n_blocks if not callable(n_blocks) else 50
        fa, la = curves(a, nb)
        fb, lb = curves(b, nb)
        d, dl = fa - fb, la - lb
        best = bracket(d, np.array([jackknife_error(dl[i]) for i in range(len(temps))]))
        if best is not None and callable(n_blocks):
            # blocks sized by the slowest of the four replicas at the bracket
            k = best[1]
            n = len(m_series[a][k])
            nb = n_blocks([m_series[a][k], m_series[a][k + 1], m_series[b][k], m_series[b][k + 1]], n)
            fa, la = curves(a, nb)
            fb, lb = curves(b, nb)
            d, dl = fa - fb, la - lb
        if best is None:
            out.append({"pair": [int(a), int(b)], "T_cross": None})
            continue
        sig, k = best
        t_star = _crossing_in(temps, d, k)
        t_loo = np.array([_crossing_in(temps, dl[:, j], k) for j in range(dl.shape[1])])
        err = jackknife_error(t_loo)
        t_quad = _crossing_quad(temps, d, k)
        syst = abs(t_quad - t_star)
        tot = math.hypot(err, syst)
        out.append({"pair": [int(a), int(b)], "T_cross": t_star, "err": err, "n_blocks": int(dl.shape[1]),
                    "bracket": [float(temps[k]), float(temps[k + 1])], "significance": float(sig),
                    "z_vs_Tc": float((t_star - T_C) / err) if err > 0 else None,
                    "T_cross_quad": t_quad, "syst": syst,
                    "z_total": float((t_star - T_C) / tot) if tot > 0 else None})
    return out
