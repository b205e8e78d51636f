"""The oracle's moments of a traced chain (Sec. 4.1: m = M / N, its square and fourth power for the
Binder cumulant, and e = E / N), pinned by traces whose sums have closed forms."""
import numpy as np
import pytest


def test_constant_trace(oracle_lib):
    N, n = 4096, 37
    tr = np.tile(np.array([[N, -2 * N]], dtype=np.int64), (n, 1))   # the ordered state
    assert oracle_lib.moments(tr, N).tolist() == [1.0, 1.0, 1.0, -2.0, 4.0]


def test_sign_of_m_drops_out_of_abs_and_even_powers(oracle_lib):
    N, n = 1024, 64
    M = np.where(np.arange(n) % 2 == 0, 256, -256)
    tr = np.stack([M, -np.full(n, 512)], axis=1).astype(np.int64)
    out = oracle_lib.moments(tr, N)
    assert out.tolist() == [0.25, 0.0625, 0.00390625, -0.5, 0.25]


@pytest.mark.parametrize("n", [1, 7, 300, 1001])
def test_linear_ramp_sums(oracle_lib, n):
    # M_k = 2k, E_k = -4k (k = 0 .. n - 1): sums of k, k^2 and k^4 in closed form
    N = 96 * 96
    k = np.arange(n, dtype=np.int64)
    tr = np.stack([2 * k, -4 * k], axis=1)
    s1 = (n - 1) * n / 2
    s2 = (n - 1) * n * (2 * n - 1) / 6
    s4 = (n - 1) * n * (2 * n - 1) * (3 * n * n - 3 * n - 1) / 30
    expect = [2 * s1 / N / n, 4 * s2 / N ** 2 / n, 16 * s4 / N ** 4 / n, -4 * s1 / N / n, 16 * s2 / N ** 2 / n]
    assert oracle_lib.moments(tr, N) == pytest.approx(expect, rel=1e-13, abs=1e-300)
