"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Integer work, so the bar is bit-exactness: every spin after every sweep and every (M, E) of
the trace.  Sizes span several 64-column groups, several row strips, ragged strip counts
(L = 192, 320) and the full 16384^2 lattice of the benchmark (checked on light-cone crops
the oracle can afford, placed on the torus seams, plus invariants).
"""
import math
import sys

import numpy as np
import pytest

from tests import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_11714_amd import ising
    ising.library()
    return ising


def _to_dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t) -> np.ndarray:
    return t.cpu().numpy()


@pytest.mark.parametrize("L,seed", [(64, 1), (128, 7), (192, 2**40 + 3), (1024, 99)])
def test_init_matches_oracle(dev, oracle_lib, L, seed):
    _say("init", L, seed)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    assert np.array_equal(_host(s), oracle_lib.init(L, seed))


def test_fill(dev):
    s = torch.zeros((128, 128), dtype=torch.int8, device="cuda")
    dev.ising_fill(s, 128, -1)
    assert (s == -1).all()
    dev.ising_fill(s, 128, 1)
    assert (s == 1).all()


@pytest.mark.parametrize("L,seed", [(64, 3), (128, 4), (320, 5)])
def test_observables_match_oracle(dev, oracle_lib, L, seed):
    _say("observables", L, seed)
    for k, host in enumerate([inputs.random_lattice(L, seed), inputs.random_lattice(L, seed + 1, 0.1),
                              inputs.all_up(L), inputs.neel(L), inputs.stripes(L, 3)]):
        s = _to_dev(host)
        out = torch.empty(2, dtype=torch.int64, device="cuda")
        dev.ising_observables(s, L, out)
        assert tuple(out.tolist()) == oracle_lib.observables(host), k


@pytest.mark.parametrize("q", [0, 1])
@pytest.mark.parametrize("L,beta", [(64, BETA_C), (128, 0.3), (192, 0.7), (256, 0.0), (128, math.inf)])
def test_half_sweep_matches_oracle(dev, oracle_lib, L, beta, q):
    _say("half_sweep", L, beta, q)
    host = inputs.random_lattice(L, seed=L + q)
    s = _to_dev(host)
    dev.ising_half_sweep(s, L, beta, 12345, 77, q)
    oracle_lib.half_sweep(host, beta, 12345, 77, q)
    assert np.array_equal(_host(s), host)


def test_config1_full_trace_bit_exact(dev, oracle_lib):
    # L = 64, seed 1, hot start, beta_c, 1000 sweeps, (M, E) after every sweep.
    L, n, seed = 64, 1000, 1
    _say("config1", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(s, L, BETA_C, n, seed, 0, trace)
    host = oracle_lib.init(L, seed)
    ref_trace = oracle_lib.sweep(host, BETA_C, n, seed, 0, trace=True)
    assert np.array_equal(_host(s), host)
    assert np.array_equal(_host(trace), ref_trace)


@pytest.mark.parametrize("L,beta,n,seed,offset", [
    (128, BETA_C, 20, 2, 0),
    (192, 0.5, 9, 3, 1000),
    (320, 0.4, 6, 2**33 + 5, 2**32 - 6),     # last valid sweep indices
    (512, 1 / 2.6, 5, 11, 17),
    (256, 0.0, 3, 1, 0),
    (256, math.inf, 4, 1, 0),
    (1024, BETA_C, 3, 8, 5),
])
def test_sweeps_match_oracle(dev, oracle_lib, L, beta, n, seed, offset):
    _say("sweeps", L, beta, n, seed, offset)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(s, L, beta, n, seed, offset, trace)
    host = oracle_lib.init(L, seed)
    ref = oracle_lib.sweep(host, beta, n, seed, offset, trace=True)
    assert np.array_equal(_host(s), host)
    assert np.array_equal(_host(trace), ref)


def test_neel_zero_temperature(dev):
    L = 128
    s = _to_dev(inputs.neel(L, white=-1))
    dev.ising_sweep(s, L, math.inf, 1, 1, 0)
    assert (s == 1).all()


def test_chunked_equals_unchunked(dev):
    L = 256
    a = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(a, L, 5)
    b = a.clone()
    dev.ising_sweep(a, L, BETA_C, 10, 5, 100)
    dev.ising_sweep(b, L, BETA_C, 3, 5, 100)
    dev.ising_sweep(b, L, BETA_C, 7, 5, 103)
    assert torch.equal(a, b)


def test_repeat_runs_identical(dev):
    L = 2048
    outs = []
    for _ in range(2):
        s = torch.empty((L, L), dtype=torch.int8, device="cuda")
        dev.ising_init(s, L, 42)
        dev.ising_sweep(s, L, BETA_C, 10, 42, 0)
        outs.append(s)
    assert torch.equal(outs[0], outs[1])


def test_full_size_16384_crops_and_invariants(dev, oracle_lib):
    # The benchmark's lattice and launch configuration: L = 16384, hot start, beta_c.
    L, n, seed = 16384, 64, 1
    _say("full-size", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(s, L, BETA_C, n, seed, 0, trace)
    torch.cuda.synchronize()
    for (r0, c0, h, w) in [(0, 0, 16, 64), (L - 8, L - 40, 16, 80), (8191, 4097, 24, 24), (100, L - 1, 5, 3)]:
        ref = oracle_lib.crop(L, seed, BETA_C, n, 0, r0, c0, h, w)
        rows = [(r0 + a) % L for a in range(h)]
        cols = [(c0 + b) % L for b in range(w)]
        got = s[rows][:, cols].cpu().numpy()
        assert np.array_equal(got, ref), (r0, c0)
    # invariants: spins stay +-1, the tracked (M, E) equals a fresh reduction
    assert bool(((s == 1) | (s == -1)).all())
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising_observables(s, L, out)
    assert out.tolist() == trace[-1].tolist()
    tr = trace.cpu().numpy()
    assert np.all(tr[:, 1] % 4 == 0) and np.all(tr[:, 0] % 2 == 0)


def test_invalid_arguments_raise(dev):
    s = torch.empty((80, 80), dtype=torch.int8, device="cuda")   # L % 32 != 0
    with pytest.raises(dev.IsingError):
        dev.ising_init(s, 80, 1)
    s = torch.empty((64, 64), dtype=torch.int8, device="cuda")
    with pytest.raises(dev.IsingError):
        dev.ising_sweep(s, 64, -1.0, 1, 1)


def test_staged_path_full_lattice_matches_oracle(dev, oracle_lib):
    # L = 4096: every wave owns 64 whole groups of a row, so rows move through LDS.
    L, n, seed = 4096, 2, 6
    _say("staged full lattice", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(s, L, BETA_C, n, seed, 3, trace)
    host = oracle_lib.init(L, seed)
    ref = oracle_lib.sweep(host, BETA_C, n, seed, 3, trace=True)
    assert np.array_equal(_host(s), host)
    assert np.array_equal(_host(trace), ref)


@pytest.mark.parametrize("L", [4096, 16384])
def test_every_launch_option_gives_identical_lattices(dev, L):
    # Launch shapes (rows per lane, XCD renumbering, LDS staging, store kind) must not change
    # a single spin: the random numbers depend only on (site, sweep, colour).  This also
    # catches races between lanes that share boundary rows.
    _say("options", L)
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, 17)
    opts = {"rows_per_lane": [0, 2, 8, 64], "xcd_remap": [1, 0], "staged": [1, 0], "nt_store": [0, 1]}
    ref = None
    try:
        for rows in opts["rows_per_lane"]:
            for remap in opts["xcd_remap"]:
                for staged in opts["staged"]:
                    for nt in opts["nt_store"]:
                        if nt and (rows, remap, staged) != (0, 1, 1):
                            continue
                        dev.ising_set_option("rows_per_lane", rows)
                        dev.ising_set_option("xcd_remap", remap)
                        dev.ising_set_option("staged", staged)
                        dev.ising_set_option("nt_store", nt)
                        s = base.clone()
                        trace = torch.empty((3, 2), dtype=torch.int64, device="cuda")
                        dev.ising_sweep(s, L, BETA_C, 3, 17, 40, trace)
                        if ref is None:
                            ref = (s, trace)
                        else:
                            assert torch.equal(s, ref[0]), (rows, remap, staged, nt)
                            assert torch.equal(trace, ref[1]), (rows, remap, staged, nt)
    finally:
        for k, v in (("rows_per_lane", 0), ("xcd_remap", 1), ("staged", 1), ("nt_store", 0)):
            dev.ising_set_option(k, v)
