"""Pin the oracle's low-precision acceptance (the paper's bfloat16 experiment, Sec. 4.1).

The paper states only that bfloat16 replaced float32 for the acceptance arithmetic.  The
reading taken: the acceptance probability exp(-2 beta s) is rounded to nearest-even in the
format, the site's 16-bit uniform chunk (the top half of its exact-chain uniform) is rounded
toward zero in the format, and the site flips when the rounded uniform is below the rounded
probability.
"""
import math

import numpy as np
import pytest
import torch

from tests import inputs


def _fp16_values():
    pats = np.arange(0, 0x3C01, dtype=np.uint16)          # +0 .. 1.0
    return np.sort(pats.view(np.float16).astype(np.float64))


def _bf16_values():
    pats = np.arange(0, 0x3F81, dtype=np.uint32) << 16      # +0 .. 1.0
    return np.sort(pats.view(np.float32).astype(np.float64))


def test_fp16_nearest_even_matches_numpy(oracle_lib):
    rng = np.random.default_rng(1)
    vals = np.concatenate([rng.random(5000), 10.0 ** rng.uniform(-9, 0, 5000),
                           np.array([2.0 ** -14, 2.0 ** -24, 3 * 2.0 ** -25, 1.0, 0.5 + 2.0 ** -12])])
    for v in vals:
        assert oracle_lib.round_fmt(v, "fp16") == float(np.float16(v)), v


def test_bf16_nearest_even_matches_torch_on_float32_inputs(oracle_lib):
    rng = np.random.default_rng(2)
    vals = np.concatenate([rng.random(5000), 10.0 ** rng.uniform(-30, 0, 3000)]).astype(np.float32)
    # ties: values exactly half-way between two bfloat16 numbers
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32) * np.float32(2.0 ** -10)
    vals = np.concatenate([vals, ties.astype(np.float32)])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle_lib.round_fmt(float(v), "bf16") for v in vals])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_uniform_rounds_toward_zero(oracle_lib, fmt):
    grid = _bf16_values() if fmt == "bf16" else _fp16_values()
    r = np.arange(65536)
    x = r / 65536.0
    expect = grid[np.searchsorted(grid, x, side="right") - 1]      # largest value <= x
    got = np.array([oracle_lib.u_fmt(int(k) << 16 | 0xBEEF, fmt) for k in r])
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_probabilities_are_nearest_representable(oracle_lib, fmt):
    grid = _bf16_values() if fmt == "bf16" else _fp16_values()
    for beta in (0.5, 0.44068679350977147, 0.4, 1 / 2.6, 0.2, 1.5):
        for s in (2, 4):
            p = math.exp(-2 * beta * s)
            got = oracle_lib.p_fmt(beta, s, fmt)
            assert got in set(grid.tolist())
            i = np.searchsorted(grid, p)
            lo, hi = grid[max(i - 1, 0)], grid[min(i, len(grid) - 1)]
            assert min(abs(p - lo), abs(p - hi)) == abs(p - got)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_lowprec_limits(oracle_lib, fmt):
    s0 = inputs.random_lattice(32, 5)
    s = s0.copy()
    oracle_lib.sweep_fmt(s, 0.0, fmt, 3, 7)             # p = 1 > every rounded uniform
    assert np.array_equal(s, -s0)
    s = inputs.neel(32, white=-1)
    oracle_lib.sweep_fmt(s, math.inf, fmt, 1, 7)        # p = 0: only s <= 0 flips
    assert (s == 1).all()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_lowprec_acceptance_frequency(oracle_lib, fmt):
    # Neel start: after the white half-sweep every black site has s = 4 and flips with
    # probability #{r : u(r) < p_4} / 2^16 (independent draws).
    L, beta = 128, 0.15
    grid = _bf16_values() if fmt == "bf16" else _fp16_values()
    p4 = oracle_lib.p_fmt(beta, 4, fmt)
    r = np.arange(65536) / 65536.0
    u = grid[np.searchsorted(grid, r, side="right") - 1]
    prob = float((u < p4).mean())
    s = inputs.neel(L, white=-1)
    oracle_lib.sweep_fmt(s, beta, fmt, 1, 31)
    black = (np.indices((L, L)).sum(axis=0) % 2 == 0)
    k = int((s[black] == -1).sum())
    n = int(black.sum())
    assert abs(k - n * prob) < 5 * math.sqrt(n * prob * (1 - prob))


def test_lowprec_chain_shares_the_exact_chains_draws(oracle_lib):
    # Same draws: the chains coincide until a site's rounded compare disagrees with the exact
    # one, which needs its uniform within a rounding step of the threshold (rare).
    s_exact = oracle_lib.init(64, 3)
    s_fp16 = s_exact.copy()
    oracle_lib.sweep(s_exact, 0.44068679350977147, 1, 3)
    oracle_lib.sweep_fmt(s_fp16, 0.44068679350977147, "fp16", 1, 3)
    diff = (s_exact != s_fp16).mean()
    assert diff < 0.01
