"""GPU parity of the low-precision acceptance form (bfloat16 / half) and of the FP64 moments.

The GPU applies the rounded comparison through exact integer thresholds; the oracle does the
literal rounded arithmetic.  Integer results, so bit-exact: every spin and every (M, E).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_11714_amd import ising
    ising.library()
    return ising


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("L,beta,n,seed", [(64, BETA_C, 200, 1), (128, 0.5, 10, 2), (320, 0.4, 5, 3),
                                           (64, 1.5, 20, 4), (128, 0.0, 3, 5)])
def test_lowprec_sweep_matches_oracle(dev, oracle_lib, fmt, L, beta, n, seed):
    print("lowprec", fmt, L, beta, n, flush=True)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fmt(s, L, beta, fmt, n, seed, 9, trace)
    host = oracle_lib.init(L, seed)
    ref = oracle_lib.sweep_fmt(host, beta, fmt, n, seed, 9, trace=True)
    assert np.array_equal(s.cpu().numpy(), host)
    assert np.array_equal(trace.cpu().numpy(), ref)


@pytest.mark.parametrize("fmt", ["exact", "bf16", "fp16"])
def test_lowprec_packed_equals_int8(dev, fmt):
    L, n = 4096, 4
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, 8)
    p = torch.empty(L * L // 32, dtype=torch.int32, device="cuda")
    dev.ising_init_packed(p, L, 8)
    t1 = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    t2 = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fmt(s, L, BETA_C, fmt, n, 8, 0, t1)
    dev.ising_sweep_packed_fmt(p, L, BETA_C, fmt, n, 8, 0, t2)
    assert torch.equal(t1, t2)
    back = torch.empty_like(s)
    dev.ising_unpack(p, L, back)
    assert torch.equal(back, s)


def test_exact_fmt_is_the_exact_chain(dev):
    L = 256
    a = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(a, L, 4)
    b = a.clone()
    dev.ising_sweep(a, L, BETA_C, 5, 4, 0)
    dev.ising_sweep_fmt(b, L, BETA_C, "exact", 5, 4, 0)
    assert torch.equal(a, b)


def test_moments_fp64_sequential(dev):
    L, n = 128, 300
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, 1)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(s, L, BETA_C, n, 1, 0, trace)
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    dev.ising_moments(trace, n, L * L, out)
    tr = trace.cpu().numpy()
    inv = 1.0 / (L * L)
    acc = [0.0] * 5
    for M, E in tr.tolist():
        m, e = M * inv, E * inv
        m2 = m * m
        acc[0] += abs(m)
        acc[1] += m2
        acc[2] += m2 * m2
        acc[3] += e
        acc[4] += e * e
    expect = [a * (1.0 / n) for a in acc]
    assert out.cpu().tolist() == expect
