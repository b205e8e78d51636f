"""GPU parity of the 1-bit packed layout: pack/unpack, hot start, observables and the sweep
against the CPU oracle (bit-exact), and packed == int8 after the same sweeps.
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


def _planes(L):
    return torch.empty(L * L // 32, dtype=torch.int32, device="cuda")


def _unpacked(dev, planes, L):
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_unpack(planes, L, s)
    return s


@pytest.mark.parametrize("L", [64, 128, 192, 4096])
def test_pack_unpack_round_trip(dev, L):
    _say("pack", L)
    host = inputs.random_lattice(L, seed=L)
    s = torch.from_numpy(host).cuda()
    p = _planes(L)
    dev.ising_pack(s, L, p)
    back = _unpacked(dev, p, L)
    assert np.array_equal(back.cpu().numpy(), host)
    # each plane word holds only its colour: half the set bits of a Neel lattice per plane
    neel = torch.from_numpy(inputs.neel(L, white=-1)).cuda()
    dev.ising_pack(neel, L, p)
    words = p.view(2, L, L // 64)
    assert bool((words[0] == 0).all())           # black = +1
    assert bool((words[1] == -1).all())          # white = -1 (all bits set)


@pytest.mark.parametrize("L,seed", [(64, 1), (320, 9), (1024, 2**35 + 1)])
def test_init_packed_matches_oracle(dev, oracle_lib, L, seed):
    p = _planes(L)
    dev.ising_init_packed(p, L, seed)
    assert np.array_equal(_unpacked(dev, p, L).cpu().numpy(), oracle_lib.init(L, seed))
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    p2 = _planes(L)
    dev.ising_pack(s, L, p2)
    assert torch.equal(p, p2)


@pytest.mark.parametrize("L", [64, 192, 512])
def test_observables_packed_match_oracle(dev, oracle_lib, L):
    for host in (inputs.random_lattice(L, 3), inputs.random_lattice(L, 4, 0.2), inputs.all_up(L),
                 inputs.neel(L), inputs.stripes(L, 5)):
        p = _planes(L)
        dev.ising_pack(torch.from_numpy(host).cuda(), L, p)
        out = torch.empty(2, dtype=torch.int64, device="cuda")
        dev.ising_observables_packed(p, L, out)
        assert tuple(out.tolist()) == oracle_lib.observables(host)


@pytest.mark.parametrize("q", [0, 1])
@pytest.mark.parametrize("L,beta", [(64, BETA_C), (192, 0.6), (256, 0.0), (128, math.inf)])
def test_half_sweep_packed_matches_oracle(dev, oracle_lib, L, beta, q):
    host = inputs.random_lattice(L, seed=3 * L + q)
    p = _planes(L)
    dev.ising_pack(torch.from_numpy(host).cuda(), L, p)
    dev.ising_half_sweep_packed(p, L, beta, 999, 12, q)
    oracle_lib.half_sweep(host, beta, 999, 12, q)
    assert np.array_equal(_unpacked(dev, p, L).cpu().numpy(), host)


@pytest.mark.parametrize("L,beta,n,seed,offset", [
    (64, BETA_C, 1000, 1, 0),          # the L = 64 trace case on the packed layout
    (128, 0.5, 12, 5, 7),
    (320, 1 / 2.6, 6, 2**34 + 9, 2**32 - 6),
    (1024, BETA_C, 3, 2, 100),
])
def test_sweep_packed_matches_oracle(dev, oracle_lib, L, beta, n, seed, offset):
    _say("packed sweeps", L, beta, n)
    p = _planes(L)
    dev.ising_init_packed(p, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_packed(p, L, beta, n, seed, offset, trace)
    host = oracle_lib.init(L, seed)
    ref = oracle_lib.sweep(host, beta, n, seed, offset, trace=True)
    assert np.array_equal(_unpacked(dev, p, L).cpu().numpy(), host)
    assert np.array_equal(trace.cpu().numpy(), ref)


@pytest.mark.parametrize("ties", [1, 0])
@pytest.mark.parametrize("L,beta,n", [(192, BETA_C, 6), (1024, 0.41, 3), (256, 0.0, 2), (128, math.inf, 2)])
def test_packed_rows_per_lane_and_tie_queue_match_oracle(dev, oracle_lib, L, beta, n, ties):
    # ties = 1: a lane decides four rows' words with two Philox blocks each and the wave settles
    # the words left with tied sites together (needs rows per lane % 4 == 0); 0: row by row
    _say("packed rows/ties", L, beta, n, ties)
    host = oracle_lib.init(L, 7)
    ref_host = host.copy()
    ref = oracle_lib.sweep(ref_host, beta, n, 7, 21, trace=True)
    try:
        dev.ising_set_option("packed_ties", ties)
        for rows in (2, 4, 8, 16, 32, 64):
            if L % rows:
                continue
            dev.ising_set_option("rows_per_lane", rows)
            p = _planes(L)
            dev.ising_pack(torch.from_numpy(host).cuda(), L, p)
            trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
            dev.ising_sweep_packed(p, L, beta, n, 7, 21, trace)
            assert np.array_equal(_unpacked(dev, p, L).cpu().numpy(), ref_host), rows
            assert np.array_equal(trace.cpu().numpy(), ref), rows
    finally:
        dev.ising_set_option("rows_per_lane", 0)
        dev.ising_set_option("packed_ties", 1)


@pytest.mark.parametrize("L,n", [(4096, 5), (16384, 8)])
def test_packed_equals_int8(dev, L, n):
    _say("packed == int8", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, 3)
    p = _planes(L)
    dev.ising_init_packed(p, L, 3)
    t8 = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    tp = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(s, L, BETA_C, n, 3, 11, t8)
    dev.ising_sweep_packed(p, L, BETA_C, n, 3, 11, tp)
    assert torch.equal(t8, tp)
    assert torch.equal(_unpacked(dev, p, L), s)


def test_full_size_16384_packed_crops(dev, oracle_lib):
    L, n, seed = 16384, 48, 1
    _say("packed full size", L, n)
    p = _planes(L)
    dev.ising_init_packed(p, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_packed(p, L, BETA_C, n, seed, 0, trace)
    s = _unpacked(dev, p, L)
    for (r0, c0, h, w) in [(0, L - 20, 12, 40), (5000, 70, 16, 16)]:
        ref = oracle_lib.crop(L, seed, BETA_C, n, 0, r0, c0, h, w)
        rows = [(r0 + a) % L for a in range(h)]
        cols = [(c0 + b) % L for b in range(w)]
        assert np.array_equal(s[rows][:, cols].cpu().numpy(), ref)
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising_observables_packed(p, L, out)
    assert out.tolist() == trace[-1].tolist()


def test_packed_at_two_to_the_nineteen(dev, oracle_lib):
    # L = 2^19: the (row, group) word count is 2^32, past any 32-bit lane index.  Fill, observables and
    # the hot start must still cover every row (32 GiB of planes).
    L = 1 << 19
    W = L // 64
    planes = torch.empty(L * L // 32, dtype=torch.int32, device="cuda")
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    for value in (1, -1):
        dev.ising_fill_packed(planes, L, value)
        dev.ising_observables_packed(planes, L, out)
        assert out.cpu().tolist() == [value * L * L, -2 * L * L]
    seed = 3
    dev.ising_init_packed(planes, L, seed)
    torch.cuda.synchronize()
    rng = np.random.default_rng(19)
    rows = np.concatenate([rng.integers(0, L, 24), [L - 1, L - 2, L // 2]])
    for r in rows.tolist():
        for q in (0, 1):
            g = int(rng.integers(0, W))
            word = int(planes[(q * L + r) * W + g].item()) & 0xFFFFFFFF
            for i in (0, 5, 17, 31):
                p = 8 * (0, 2, 1, 3)[i & 3] + (i >> 2)
                c = 2 * (32 * g + i) + ((r + q) & 1)
                spin = -1 if (word >> p) & 1 else 1
                assert spin == oracle_lib.init_site(seed, r, c), (r, q, g, i)
    del planes
    torch.cuda.empty_cache()
