"""GPU parity of the 3-D sweep (L x L x L torus, six neighbours) against the CPU oracle.

Integer work, so the bar is bit-exactness: every spin and every traced (M, E).  Sizes cover
workgroups that hold whole planes (L = 64, 128: y wraps inside the workgroup), workgroups of a
few rows that take their outer rows from the neighbouring strip (L = 256, 512, 1024, 2048, with
4 and 8 waves), every plane count per workgroup, and the limits beta = 0 and zero temperature.
Lattices above 256^3 are checked on light-cone blocks across the torus seams.  The 1-bit layout is
checked against the oracle and, spin for spin, against the int8 layout.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

BETA_C3 = 0.2216546  # simple-cubic critical coupling (Monte Carlo estimate; only a test temperature)


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


def _cube(L, seed, p_down=0.5):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L, L)) < p_down, -1, 1).astype(np.int8)


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _parity(L):
    z, y, x = np.indices((L, L, L))
    return (x + y + z) & 1


@pytest.mark.parametrize("L,seed", [(64, 1), (128, 2**40 + 5), (256, 3)])
def test_init3_matches_oracle(dev, oracle_lib, L, seed):
    _say("init3", L)
    s = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_init(s, L, seed)
    assert np.array_equal(s.cpu().numpy(), oracle_lib.init3(L, seed))


@pytest.mark.parametrize("L", [64, 128, 256])
def test_observables3_match_oracle(dev, oracle_lib, L):
    _say("observables3", L)
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    for host in (_cube(L, L), _cube(L, L + 1, 0.1), np.ones((L, L, L), dtype=np.int8),
                 np.where(_parity(L) == 0, 1, -1).astype(np.int8)):
        dev.ising3_observables(_to_dev(host), L, out)
        assert tuple(out.tolist()) == oracle_lib.observables3(host)


@pytest.mark.parametrize("q", [1, 0])
@pytest.mark.parametrize("L,beta", [(64, BETA_C3), (128, 0.15), (256, 0.3), (256, 0.0), (128, math.inf)])
def test_half_sweep3_matches_oracle(dev, oracle_lib, L, beta, q):
    _say("half_sweep3", L, beta, q)
    host = _cube(L, 7 * L + q)
    s = _to_dev(host)
    dev.ising3_half_sweep(s, L, beta, 99, 13, q)
    oracle_lib.half_sweep3(host, beta, 99, 13, q)
    assert np.array_equal(s.cpu().numpy(), host)


@pytest.mark.parametrize("ties", [1, 0])
@pytest.mark.parametrize("L,beta,n,seed,offset", [(64, BETA_C3, 10, 1, 0), (128, 0.25, 4, 2**33 + 1, 7),
                                                  (256, BETA_C3, 2, 5, 2**32 - 2), (128, 0.0, 2, 3, 0),
                                                  (64, math.inf, 2, 4, 1)])
def test_sweeps3_match_oracle(dev, oracle_lib, L, beta, n, seed, offset, ties):
    # ties = 1: the two planes of each step share one exchange and one tie queue; 0: plane by plane
    _say("sweep3", L, beta, n, ties)
    s = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_init(s, L, seed)
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_set_option("ties3", ties)
    try:
        dev.ising3_sweep(s, L, beta, n, seed, offset, tr)
    finally:
        dev.ising_set_option("ties3", 1)
    host = oracle_lib.init3(L, seed)
    ref = oracle_lib.sweep3(host, beta, n, seed, offset, trace=True)
    assert np.array_equal(s.cpu().numpy(), host)
    assert np.array_equal(tr.cpu().numpy(), ref)


def test_limits3(dev):
    L = 128
    s0 = torch.from_numpy(_cube(L, 9)).cuda()
    s = s0.clone()
    dev.ising3_sweep(s, L, 0.0, 1, 4)               # beta = 0: every site flips
    assert torch.equal(s, -s0)
    s = _to_dev(np.where(_parity(L) == 0, 1, -1).astype(np.int8))
    dev.ising3_sweep(s, L, math.inf, 1, 4)          # white sites see six anti-aligned neighbours
    assert bool((s == 1).all())


@pytest.mark.parametrize("L,n", [(512, 4), (1024, 3), (2048, 2)])
def test_large3_light_cone_blocks(dev, oracle_lib, L, n):
    seed, beta = 1, BETA_C3
    _say("large3", L, n)
    s = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_init(s, L, seed)
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising3_sweep(s, L, beta, n, seed, 0, tr)
    torch.cuda.synchronize()
    for (z0, y0, x0, d, h, w) in [(L - 6, L - 5, L - 40, 12, 10, 80), (L // 2 + 3, 17, 100, 8, 9, 70)]:
        ref = oracle_lib.crop3(L, seed, beta, n, 0, z0, y0, x0, d, h, w)
        zz = torch.tensor([(z0 + a) % L for a in range(d)], device="cuda")
        yy = torch.tensor([(y0 + a) % L for a in range(h)], device="cuda")
        xx = torch.tensor([(x0 + a) % L for a in range(w)], device="cuda")
        got = s.index_select(0, zz).index_select(1, yy).index_select(2, xx).cpu().numpy()
        assert np.array_equal(got, ref), (z0, y0, x0)
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising3_observables(s, L, out)
    assert out.tolist() == tr[-1].tolist()
    assert bool(((s == 1) | (s == -1)).all())
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L", [256, 512])
def test_every_plane_count_gives_identical_lattices(dev, L):
    _say("planes3", L)
    base = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_init(base, L, 17)
    ref = None
    try:
        for rz in (0, 2, 4, 8, 16, 32, 64):
            for remap, ties in ((1, 1), (0, 1), (1, 0)):
                dev.ising_set_option("planes3", rz)
                dev.ising_set_option("xcd_remap", remap)
                dev.ising_set_option("ties3", ties)
                s = base.clone()
                tr = torch.empty((3, 2), dtype=torch.int64, device="cuda")
                dev.ising3_sweep(s, L, BETA_C3, 3, 17, 40, tr)
                if ref is None:
                    ref = (s, tr)
                else:
                    assert torch.equal(s, ref[0]), (rz, remap, ties)
                    assert torch.equal(tr, ref[1]), (rz, remap, ties)
    finally:
        dev.ising_set_option("planes3", 0)
        dev.ising_set_option("xcd_remap", 1)
        dev.ising_set_option("ties3", 1)


def test_invalid_3d_arguments_raise(dev):
    s = torch.empty(96 ** 3, dtype=torch.int8, device="cuda")
    with pytest.raises(dev.IsingError):
        dev.ising3_init(s, 96, 1)
    s = torch.empty(64 ** 3, dtype=torch.int8, device="cuda")
    with pytest.raises(dev.IsingError):
        dev.ising3_sweep(s, 64, -0.5, 1, 1)


# ---- 1-bit layout of the cubic lattice ----------------------------------------------------------

def _planes3(L):
    return torch.empty(L ** 3 // 32, dtype=torch.int32, device="cuda")


def _unpacked3(dev, p, L):
    s = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_unpack(p, L, s)
    return s


@pytest.mark.parametrize("L", [64, 128, 256])
def test_pack3_round_trip_and_packed_hot_start(dev, oracle_lib, L):
    _say("pack3", L)
    host = _cube(L, 3 * L)
    p = _planes3(L)
    dev.ising3_pack(_to_dev(host), L, p)
    assert np.array_equal(_unpacked3(dev, p, L).cpu().numpy(), host)
    dev.ising3_init_packed(p, L, 77)
    assert np.array_equal(_unpacked3(dev, p, L).cpu().numpy(), oracle_lib.init3(L, 77))
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising3_observables_packed(p, L, out)
    assert tuple(out.tolist()) == oracle_lib.observables3(oracle_lib.init3(L, 77))


@pytest.mark.parametrize("q", [1, 0])
@pytest.mark.parametrize("L,beta", [(64, BETA_C3), (128, 0.15), (256, 0.0), (128, math.inf)])
def test_half_sweep3_packed_matches_oracle(dev, oracle_lib, L, beta, q):
    _say("half_sweep3_packed", L, beta, q)
    host = _cube(L, 11 * L + q)
    p = _planes3(L)
    dev.ising3_pack(_to_dev(host), L, p)
    dev.ising3_half_sweep_packed(p, L, beta, 99, 13, q)
    oracle_lib.half_sweep3(host, beta, 99, 13, q)
    assert np.array_equal(_unpacked3(dev, p, L).cpu().numpy(), host)


@pytest.mark.parametrize("L,beta,n,seed,offset", [(64, BETA_C3, 10, 1, 0), (128, 0.25, 4, 2**33 + 1, 7)])
def test_sweeps3_packed_match_oracle(dev, oracle_lib, L, beta, n, seed, offset):
    _say("sweep3_packed", L, n)
    p = _planes3(L)
    dev.ising3_init_packed(p, L, seed)
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising3_sweep_packed(p, L, beta, n, seed, offset, tr)
    host = oracle_lib.init3(L, seed)
    ref = oracle_lib.sweep3(host, beta, n, seed, offset, trace=True)
    assert np.array_equal(_unpacked3(dev, p, L).cpu().numpy(), host)
    assert np.array_equal(tr.cpu().numpy(), ref)


@pytest.mark.parametrize("ties", [1, 0])
@pytest.mark.parametrize("L,beta,n", [(64, BETA_C3, 3), (128, 0.15, 2), (64, 0.0, 1), (64, math.inf, 2)])
def test_packed3_planes_and_tie_queue_match_oracle(dev, oracle_lib, L, beta, n, ties):
    # ties = 1: a lane decides four planes' words with two Philox blocks each and the wave settles
    # the words left with tied sites together (needs planes per lane % 4 == 0); 0: plane by plane
    _say("packed3 planes/ties", L, beta, n, ties)
    host = oracle_lib.init3(L, 5)
    ref_host = host.copy()
    ref = oracle_lib.sweep3(ref_host, beta, n, 5, 9, trace=True)
    try:
        dev.ising_set_option("packed_ties", ties)
        for rz in (2, 4, 8, 16, 32):
            dev.ising_set_option("planes3", rz)
            p = _planes3(L)
            dev.ising3_pack(_to_dev(host), L, p)
            tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
            dev.ising3_sweep_packed(p, L, beta, n, 5, 9, tr)
            assert np.array_equal(_unpacked3(dev, p, L).cpu().numpy(), ref_host), rz
            assert np.array_equal(tr.cpu().numpy(), ref), rz
    finally:
        dev.ising_set_option("planes3", 0)
        dev.ising_set_option("packed_ties", 1)


@pytest.mark.parametrize("ties", [1, 0])
def test_sweeps3_packed_trace_across_folds(dev, oracle_lib, ties):
    # With the tie queue, the first launch of sweep i + 1 counts (M, E) after sweep i and an
    # observables pass counts the last sweep's; without it the second launch of each sweep counts.
    # 70 traced sweeps span a fold of the 64 spread sets; a second call of one sweep continues the
    # chain, and a call of no sweeps leaves lattice and trace untouched.
    L, n, seed = 64, 70, 21
    _say("sweep3_packed across folds", L, n, ties)
    host = oracle_lib.init3(L, seed)
    ref = oracle_lib.sweep3(host, BETA_C3, n, seed, 0, trace=True)
    ref1 = oracle_lib.sweep3(host, BETA_C3, 1, seed, n, trace=True)
    try:
        dev.ising_set_option("packed_ties", ties)
        p = _planes3(L)
        dev.ising3_init_packed(p, L, seed)
        tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        dev.ising3_sweep_packed(p, L, BETA_C3, n, seed, 0, tr)
        assert np.array_equal(tr.cpu().numpy(), ref)
        dev.ising3_sweep_packed(p, L, BETA_C3, 0, seed, n, torch.empty((0, 2), dtype=torch.int64, device="cuda"))
        t1 = torch.full((1, 2), -7, dtype=torch.int64, device="cuda")
        dev.ising3_sweep_packed(p, L, BETA_C3, 1, seed, n, t1)
        assert np.array_equal(t1.cpu().numpy(), ref1)
        assert np.array_equal(_unpacked3(dev, p, L).cpu().numpy(), host)
    finally:
        dev.ising_set_option("packed_ties", 1)


@pytest.mark.parametrize("L,n", [(256, 3), (1024, 2)])
def test_packed3_equals_int8(dev, L, n):
    _say("packed3 == int8", L, n)
    s = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_init(s, L, 8)
    p = _planes3(L)
    dev.ising3_init_packed(p, L, 8)
    t8 = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    tp = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising3_sweep(s, L, BETA_C3, n, 8, 3, t8)
    dev.ising3_sweep_packed(p, L, BETA_C3, n, 8, 3, tp)
    assert torch.equal(t8, tp)
    assert torch.equal(_unpacked3(dev, p, L), s)
    del s, p
    torch.cuda.empty_cache()


# ---- both colours in one pass, out of place -----------------------------------------------------

@pytest.mark.parametrize("L,beta,n,seed,offset", [(64, BETA_C3, 1, 1, 0), (64, BETA_C3, 6, 2, 5),
                                                  (128, 0.25, 4, 3, 0), (256, BETA_C3, 3, 2**40 + 3, 11),
                                                  (256, 0.0, 2, 9, 0), (128, math.inf, 2, 10, 2**32 - 2)])
@pytest.mark.parametrize("ties", [1, 0])
def test_fused3_sweeps_match_oracle(dev, oracle_lib, L, beta, n, seed, offset, ties):
    # ties = 1: the pass that updates the white sites of planes z, z + 1 and the black sites of
    # planes z - 3, z - 2 in one step and settles their tied words together; ties = 0: white sites of
    # plane z, then black sites of plane z - 1, each word on its own
    _say("fused3", L, beta, n, ties)
    host = _cube(L, L + n)
    s, scratch = _to_dev(host), torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    try:
        dev.ising_set_option("ties3", ties)
        dev.ising3_sweep_fused(s, scratch, L, beta, n, seed, offset, tr)
    finally:
        dev.ising_set_option("ties3", 1)
    ref = oracle_lib.sweep3(host, beta, n, seed, offset, trace=True)
    assert np.array_equal(s.cpu().numpy(), host)
    assert np.array_equal(tr.cpu().numpy(), ref)


@pytest.mark.parametrize("L,n", [(128, 3), (256, 2)])
def test_fused3_short_walks_match_oracle(dev, oracle_lib, L, n):
    # walks of 2, 4 and 16 planes per workgroup: the first and last steps of a walk make only some of
    # their plane updates, and with 2 planes no step has all of them (128^3: whole planes per
    # workgroup; 256^3: row strips with halo rows)
    host0 = _cube(L, 3 * L + n)
    ref = host0.copy()
    ref_tr = oracle_lib.sweep3(ref, BETA_C3, n, 77, 9, trace=True)
    scratch = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    try:
        for rz in (2, 4, 16):
            for ties in (1, 0):
                _say("fused3 short walk", L, n, rz, ties)
                dev.ising_set_option("planes3", rz)
                dev.ising_set_option("ties3", ties)
                s = _to_dev(host0)
                tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
                dev.ising3_sweep_fused(s, scratch, L, BETA_C3, n, 77, 9, tr)
                assert np.array_equal(s.cpu().numpy(), ref), (rz, ties)
                assert np.array_equal(tr.cpu().numpy(), ref_tr), (rz, ties)
    finally:
        dev.ising_set_option("planes3", 0)
        dev.ising_set_option("ties3", 1)


@pytest.mark.parametrize("L", [64, 256, 512])
def test_fused3_step_is_one_sweep_out_of_place(dev, oracle_lib, L):
    _say("fused3 step", L)
    host = oracle_lib.init3(L, 21)
    src = _to_dev(host)
    keep = src.clone()
    dst = torch.empty_like(src)
    me = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising3_sweep_fused_step(src, dst, L, BETA_C3, 21, 7, me)
    oracle_lib.sweep3(host, BETA_C3, 1, 21, 7)
    assert torch.equal(src, keep)
    assert np.array_equal(dst.cpu().numpy(), host)
    assert tuple(me.tolist()) == oracle_lib.observables3(host)


@pytest.mark.parametrize("L,n", [(512, 4), (1024, 3), (2048, 2)])
def test_fused3_equals_two_pass_for_every_plane_count(dev, L, n):
    # the two-pass sweep is pinned to the oracle at these sizes (light-cone blocks above); the fused
    # pass must give the same lattice and trace for every plane count per workgroup
    _say("fused3 == two-pass", L, n)
    base = torch.empty((L, L, L), dtype=torch.int8, device="cuda")
    dev.ising3_init(base, L, 5)
    ref = base.clone()
    ref_tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising3_sweep(ref, L, BETA_C3, n, 5, 30, ref_tr)
    scratch = torch.empty_like(base)
    try:
        for rz in ((0, 2, 8, 32) if L <= 1024 else (0, 16)):
            for remap, ties in ((1, 1), (0, 1), (1, 0)):
                dev.ising_set_option("planes3", rz)
                dev.ising_set_option("xcd_remap", remap)
                dev.ising_set_option("ties3", ties)
                s = base.clone()
                tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
                dev.ising3_sweep_fused(s, scratch, L, BETA_C3, n, 5, 30, tr)
                assert torch.equal(s, ref), (rz, remap, ties)
                assert torch.equal(tr, ref_tr), (rz, remap, ties)
    finally:
        dev.ising_set_option("planes3", 0)
        dev.ising_set_option("xcd_remap", 1)
        dev.ising_set_option("ties3", 1)
    del base, ref, scratch
    torch.cuda.empty_cache()


def test_fused3_rejects_overlap(dev):
    L = 64
    s = torch.empty(2 * L ** 3, dtype=torch.int8, device="cuda")
    with pytest.raises(dev.IsingError):
        dev.ising3_sweep_fused(s[:L ** 3], s[L ** 3 - 16:2 * L ** 3 - 16], L, BETA_C3, 2, 1)
