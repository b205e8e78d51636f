"""Exact results for the periodic 2D Ising model (J = 1, no field), used to pin the oracle.

TEST INFRASTRUCTURE ONLY.

* ``enumerate_states``: every configuration of a small L x L torus, with its energy and
  magnetisation, straight from the Hamiltonian of Sec. 3 (each bond counted once).
* ``boltzmann_moments``: exact Boltzmann averages (Sec. 3, <f> = sum f pi) from that list.
* ``kaufman_log_z``: Kaufman's (1949) closed form of the finite-torus partition function,
  an independent route to the same numbers.
* ``onsager_energy`` / ``yang_magnetisation``: the infinite-lattice energy per site
  (Onsager 1944) and spontaneous magnetisation (Yang 1952).
* ``BETA_C``: the critical point, T_c = 2 / ln(1 + sqrt 2) (Sec. 4.1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ellipk

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))
T_C = 1.0 / BETA_C


def enumerate_states(L: int):
    """Return (E, M) int64 arrays over all 2^(L*L) states of the L x L torus.

    State index b encodes site (r, c) = bit r*L + c; a set bit is spin -1.
    """
    n = L * L
    if n > 20:
        raise ValueError("enumeration is only meant for tiny lattices")
    idx = np.arange(1 << n, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    spins = (1 - 2 * bits).reshape(-1, L, L).astype(np.int64)
    M = spins.sum(axis=(1, 2))
    E = -(spins * np.roll(spins, -1, axis=2)).sum(axis=(1, 2)) \
        - (spins * np.roll(spins, -1, axis=1)).sum(axis=(1, 2))
    return E, M


def enumerate_states3(L: int):
    """Return (E, M) int64 arrays over all 2^(L^3) states of the L x L x L torus (tiny L only).

    E = -sum over every site of sigma (sigma_{x+1} + sigma_{y+1} + sigma_{z+1}): each bond once,
    so on the L = 2 torus the two bonds between a pair of sites both count.
    """
    n = L ** 3
    if n > 20:
        raise ValueError("enumeration is only meant for tiny lattices")
    idx = np.arange(1 << n, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    spins = (1 - 2 * bits).reshape(-1, L, L, L).astype(np.int64)
    M = spins.sum(axis=(1, 2, 3))
    E = -sum((spins * np.roll(spins, -1, axis=ax)).sum(axis=(1, 2, 3)) for ax in (1, 2, 3))
    return E, M


def boltzmann_moments3(L: int, beta: float) -> dict[str, float]:
    """Exact <E>/N, <|M|>/N, <M^2>/N^2, <M^4>/N^4 and U4 of the L x L x L torus."""
    E, M = enumerate_states3(L)
    N = L ** 3
    w = -beta * E.astype(np.float64)
    p = np.exp(w - w.max())
    p /= p.sum()
    m = M.astype(np.float64) / N
    m2 = float((p * m * m).sum())
    m4 = float((p * m ** 4).sum())
    return {"e": float((p * E).sum()) / N, "abs_m": float((p * np.abs(m)).sum()), "m2": m2, "m4": m4,
            "U4": 1.0 - m4 / (3.0 * m2 * m2)}


def density_of_states(L: int) -> dict[int, int]:
    E, _ = enumerate_states(L)
    vals, counts = np.unique(E, return_counts=True)
    return {int(v): int(c) for v, c in zip(vals, counts)}


def boltzmann_moments(L: int, beta: float) -> dict[str, float]:
    """Exact <E>/N, <|M|>/N, <M^2>/N^2, <M^4>/N^4, U4 and ln Z of the L x L torus."""
    E, M = enumerate_states(L)
    N = L * L
    w = -beta * E.astype(np.float64)
    wmax = w.max()
    p = np.exp(w - wmax)
    Z = p.sum()
    p /= Z
    m = M.astype(np.float64) / N
    m2 = float((p * m * m).sum())
    m4 = float((p * m ** 4).sum())
    return {
        "e": float((p * E).sum()) / N,
        "abs_m": float((p * np.abs(m)).sum()),
        "m2": m2,
        "m4": m4,
        "U4": 1.0 - m4 / (3.0 * m2 * m2),
        "e2": float((p * (E.astype(np.float64) / N) ** 2).sum()),
        "log_z": float(math.log(Z) + wmax),
    }


def kaufman_log_z(beta: float, m: int, n: int) -> float:
    """ln Z of the m x n periodic lattice from Kaufman's closed form.

    Z = 1/2 (2 sinh 2K)^(mn/2) (Z1 + Z2 + Z3 + Z4), with
    Z1 = prod_r 2 cosh(m g_{2r+1} / 2), Z2 = prod_r 2 sinh(m g_{2r+1} / 2),
    Z3 = prod_r 2 cosh(m g_{2r} / 2),   Z4 = prod_r 2 sinh(m g_{2r} / 2), r = 0..n-1,
    cosh g_k = cosh 2K coth 2K - cos(pi k / n) for k != 0 and g_0 = 2K + ln tanh K.
    """
    K = beta
    c2 = math.cosh(2 * K) * (math.cosh(2 * K) / math.sinh(2 * K))

    def gamma(k: int) -> float:
        if k == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c2 - math.cos(math.pi * k / n))

    odd = [gamma(2 * r + 1) for r in range(n)]
    even = [gamma(2 * r) for r in range(n)]
    z1 = math.prod(2 * math.cosh(m * g / 2) for g in odd)
    z2 = math.prod(2 * math.sinh(m * g / 2) for g in odd)
    z3 = math.prod(2 * math.cosh(m * g / 2) for g in even)
    z4 = math.prod(2 * math.sinh(m * g / 2) for g in even)
    return math.log(0.5) + (m * n / 2) * math.log(2 * math.sinh(2 * K)) + math.log(z1 + z2 + z3 + z4)


def onsager_energy(beta: float) -> float:
    """Energy per site of the infinite lattice: -coth 2K [1 + (2/pi)(2 tanh^2 2K - 1) K(k)],
    k = 2 sinh 2K / cosh^2 2K (scipy's ellipk takes the parameter k^2)."""
    K = beta
    k = 2 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    factor = 2 * math.tanh(2 * K) ** 2 - 1
    if abs(factor) < 1e-15:      # at T_c the logarithmic divergence of K(k) is multiplied by 0
        return -1.0 / math.tanh(2 * K)
    kk = float(ellipk(k * k))
    return -(1.0 / math.tanh(2 * K)) * (1 + (2 / math.pi) * factor * kk)


def yang_magnetisation(beta: float) -> float:
    """Spontaneous magnetisation (1 - sinh^-4 2K)^(1/8) below T_c, 0 above."""
    if beta <= BETA_C:
        return 0.0
    return (1.0 - math.sinh(2 * beta) ** -4) ** 0.125
