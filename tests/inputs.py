"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no arithmetic of the method: only lattices of given structure and seeded parameter
draws.  The hot start itself (a Philox-defined initial state) is part of the method and is
implemented separately by the oracle and by the HIP path.
"""
from __future__ import annotations

import numpy as np


def random_lattice(L: int, seed: int, p_minus: float = 0.5) -> np.ndarray:
    """iid +-1 spins, P(-1) = p_minus, from numpy's PCG64 stream `seed`."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L)) < p_minus, -1, 1).astype(np.int8)


def all_up(L: int) -> np.ndarray:
    return np.ones((L, L), dtype=np.int8)


def neel(L: int, white: int = -1) -> np.ndarray:
    """Checkerboard state: sites with (r + c) odd ("white") hold `white`, the others -white."""
    r, c = np.indices((L, L))
    return np.where((r + c) % 2 == 1, white, -white).astype(np.int8)


def stripes(L: int, width: int) -> np.ndarray:
    """Vertical stripes of alternating sign, `width` columns each."""
    c = np.arange(L)
    row = np.where((c // width) % 2 == 0, 1, -1).astype(np.int8)
    return np.tile(row, (L, 1))


def seeds(n: int, base: int = 1) -> list[int]:
    return [base + i for i in range(n)]
