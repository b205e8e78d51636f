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
    # the FP64 moments of a traced chain equal the oracle's plain sums in sweep order, bit for bit
    # (same operations in the same order: M / N, products, sums, one division by n)
    import oracle
    for L, n in ((128, 300), (96, 257)):
        s = torch.empty((L, L), dtype=torch.int8, device="cuda")
        trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        if L % 64 == 0:
            dev.ising_init(s, L, 1)
            dev.ising_sweep(s, L, BETA_C, n, 1, 0, trace)
        else:
            # any int64 trace will do: a seeded one within the (M, E) range of an L x L lattice
            rng = np.random.default_rng(L)
            tr = np.stack([rng.integers(-L * L, L * L + 1, n), rng.integers(-2 * L * L, 2 * L * L + 1, n)], axis=1)
            trace.copy_(torch.from_numpy(tr.astype(np.int64)))
        out = torch.empty(5, dtype=torch.float64, device="cuda")
        dev.ising_moments(trace, n, L * L, out)
        expect = oracle.moments(trace.cpu().numpy(), L * L)
        assert out.cpu().numpy().tolist() == expect.tolist(), (L, n)