"""Exact results for the periodic 2D Ising model (J = 1, no field), used to pin the oracle.

TEST INFRASTRUCTURE ONLY.

* ``enumerate_states``: every configuration of a small L x L torus, with its energy and
  magnetisation, straight from the Hamiltonian of Sec. 3 (each bond counted once).
* ``boltzmann_moments``: exact Boltzmann averages (Sec. 3, <f> = sum f pi) from that list.
* ``kaufman_log_z``: Kaufman's (1949) closed form of the finite-torus partition function,
  an independent route to the same numbers.
* ``BETA_C``: the critical point, T_c = 2 / ln(1 + sqrt 2) (Sec. 4.1).
"""
from __future__ import annotations

import math

import numpy as np

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
    The products are summed as logarithms with their signs (g_0 < 0 above T_c makes Z4 negative),
    so large lattices do not overflow.
    """
    K = beta
    c2 = math.cosh(2 * K) * (math.cosh(2 * K) / math.sinh(2 * K))

    def gamma(k: int) -> float:
        if k == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c2 - math.cos(math.pi * k / n))

    def log_prod(gs, hyper):
        """(log |prod 2 hyper(m g / 2)|, sign of the product)."""
        total, sign = 0.0, 1.0
        for g in gs:
            x = m * g / 2
            ax = abs(x)
            if hyper == "cosh":
                total += ax + math.log1p(math.exp(-2 * ax))
            else:
                if x == 0:
                    return -math.inf, 0.0
                total += ax + math.log1p(-math.exp(-2 * ax))
                sign *= 1.0 if x > 0 else -1.0
        return total, sign

    odd = [gamma(2 * r + 1) for r in range(n)]
    even = [gamma(2 * r) for r in range(n)]
    terms = [log_prod(odd, "cosh"), log_prod(odd, "sinh"), log_prod(even, "cosh"), log_prod(even, "sinh")]
    top = max(t for t, s in terms if s != 0.0)
    acc = sum(s * math.exp(t - top) for t, s in terms if s != 0.0)
    return math.log(0.5) + (m * n / 2) * math.log(2 * math.sinh(2 * K)) + top + math.log(acc)
