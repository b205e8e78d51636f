"""GPU parity of the fused sweep (both colours in one pass, out of place) against the CPU oracle.

The fused pass reads one buffer and writes the other; every decision uses the site's own uniform,
so the lattice and the (M, E) trace must equal the oracle's two half-sweeps bit for bit.  Cases:
one workgroup thread per 64-column group with threads past the last group idle (L = 64, 192,
320), whole waves staged through LDS (L = 4096, 8192), the full 16384^2 benchmark lattice, the
largest full-row lattice (65536^2, 1024 threads per workgroup, rows forced by option) and the
column-band pass, the default above L = 16384; the two-sweep pass with two steps' ties settled
together (rows of up to 512 groups, the default there) and with one step's.
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


@pytest.mark.parametrize("ties,pairs", [(1, 1), (1, 0), (0, 0)])
@pytest.mark.parametrize("fmt", ["exact", "bf16", "fp16"])
@pytest.mark.parametrize("L,beta,n,seed,offset", [
    (64, BETA_C, 1, 1, 0), (64, BETA_C, 6, 2, 5), (128, 0.3, 4, 3, 0), (192, 0.7, 5, 2**40 + 3, 11),
    (320, 1 / 2.6, 2, 8, 1000), (256, 0.0, 3, 9, 0), (128, math.inf, 4, 10, 2**32 - 4)])
def test_fused_sweeps_match_oracle(dev, oracle_lib, L, beta, n, seed, offset, fmt, ties, pairs):
    # ties: the fused passes settle the still-tied words of a step's updates together (1) or each
    # update finishes its own words (0); pairs: the two-sweep pass settles two steps' words together
    _say("fused", L, beta, n, seed, offset, fmt, ties, pairs)
    host = inputs.random_lattice(L, seed=L + n)
    s, scratch = _to_dev(host), torch.empty((L, L), dtype=torch.int8, device="cuda")
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_set_option("fused_ties", ties)
    dev.ising_set_option("fused_pairs", pairs)
    try:
        dev.ising_sweep_fused(s, scratch, L, beta, fmt, n, seed, offset, trace)
    finally:
        dev.ising_set_option("fused_ties", 1)
        dev.ising_set_option("fused_pairs", 1)
    if fmt == "exact":
        ref = oracle_lib.sweep(host, beta, n, seed, offset, trace=True)
    else:
        ref = oracle_lib.sweep_fmt(host, beta, fmt, n, seed, offset, trace=True)
    assert np.array_equal(s.cpu().numpy(), host)
    assert np.array_equal(trace.cpu().numpy(), ref)


@pytest.mark.parametrize("L", [64, 192, 4096])
def test_fused_step_is_one_sweep_out_of_place(dev, oracle_lib, L):
    _say("fused step", L)
    host = oracle_lib.init(L, 21)
    src = _to_dev(host)
    keep = src.clone()
    dst = torch.empty_like(src)
    me = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused_step(src, dst, L, BETA_C, "exact", 21, 7, me)
    oracle_lib.sweep(host, BETA_C, 1, 21, 7)
    assert torch.equal(src, keep)
    assert np.array_equal(dst.cpu().numpy(), host)
    assert tuple(me.tolist()) == oracle_lib.observables(host)


@pytest.mark.parametrize("L,n", [(4096, 2), (8192, 1)])
def test_fused_staged_full_lattice_matches_oracle(dev, oracle_lib, L, n):
    _say("fused staged", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, 6)
    scratch = torch.empty_like(s)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused(s, scratch, L, BETA_C, "exact", n, 6, 3, trace)
    host = oracle_lib.init(L, 6)
    ref = oracle_lib.sweep(host, BETA_C, n, 6, 3, trace=True)
    assert np.array_equal(s.cpu().numpy(), host)
    assert np.array_equal(trace.cpu().numpy(), ref)


@pytest.mark.parametrize("L", [192, 4096, 16384])
def test_fused_equals_two_half_sweeps_for_every_strip_height(dev, L):
    # Strip heights and walking directions change which rows each workgroup recomputes and in
    # which order; none may change a spin.
    _say("fused strips", L)
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, 17)
    ref = base.clone()
    ref_tr = torch.empty((4, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fmt(ref, L, BETA_C, "exact", 4, 17, 40, ref_tr)
    scratch = torch.empty_like(base)
    try:
        for sweeps, ties, pairs in ((1, 0, 1), (1, 1, 1), (2, 0, 1), (2, 1, 0), (2, 1, 1)):
            dev.ising_set_option("fused_sweeps", sweeps)
            dev.ising_set_option("fused_ties", ties)
            dev.ising_set_option("fused_pairs", pairs)
            for rows in (0, 2, 4, 8, 16, 32, 64, 128, 256):
                if rows and (L % rows or rows > L):
                    continue
                for remap, staged, alt in ((1, 1, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0), (0, 0, 0)):
                    dev.ising_set_option("fused_rows", rows)
                    dev.ising_set_option("xcd_remap", remap)
                    dev.ising_set_option("staged", staged)
                    dev.ising_set_option("fused_alternate", alt)
                    s = base.clone()
                    tr = torch.empty((4, 2), dtype=torch.int64, device="cuda")
                    dev.ising_sweep_fused(s, scratch, L, BETA_C, "exact", 4, 17, 40, tr)
                    assert torch.equal(s, ref), (sweeps, ties, pairs, rows, remap, staged, alt)
                    assert torch.equal(tr, ref_tr), (sweeps, ties, pairs, rows, remap, staged, alt)
    finally:
        for k, v in (("fused_rows", 0), ("xcd_remap", 1), ("staged", 1), ("fused_alternate", 1), ("fused_sweeps", 2),
                     ("fused_ties", 1), ("fused_pairs", 1)):
            dev.ising_set_option(k, v)


@pytest.mark.parametrize("L", [192, 4096])
def test_fused_sweep_counts_with_one_and_two_sweeps_per_pass(dev, L):
    # every count splits into passes of one or two sweeps that end in the caller's buffer
    _say("fused counts", L)
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, 23)
    scratch = torch.empty_like(base)
    try:
        for n in range(0, 8):
            ref = base.clone()
            ref_tr = torch.empty((max(n, 1), 2), dtype=torch.int64, device="cuda")
            dev.ising_sweep_fmt(ref, L, 0.41, "exact", n, 23, 9, ref_tr[:n])
            for sweeps, ties in ((1, 0), (1, 1), (2, 0), (2, 1)):
                dev.ising_set_option("fused_sweeps", sweeps)
                dev.ising_set_option("fused_ties", ties)
                s = base.clone()
                tr = torch.empty((max(n, 1), 2), dtype=torch.int64, device="cuda")
                dev.ising_sweep_fused(s, scratch, L, 0.41, "exact", n, 23, 9, tr[:n])
                assert torch.equal(s, ref), (n, sweeps, ties)
                assert torch.equal(tr[:n], ref_tr[:n]), (n, sweeps, ties)
    finally:
        dev.ising_set_option("fused_sweeps", 2)
        dev.ising_set_option("fused_ties", 1)


@pytest.mark.parametrize("L,fmt", [(64, "exact"), (192, "bf16"), (4096, "exact")])
def test_fused_pair_is_two_sweeps_out_of_place(dev, oracle_lib, L, fmt):
    _say("fused pair", L, fmt)
    host = oracle_lib.init(L, 31)
    src = _to_dev(host)
    keep = src.clone()
    dst = torch.empty_like(src)
    me = torch.empty((2, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused_pair(src, dst, L, BETA_C, fmt, 31, 12, me)
    if fmt == "exact":
        ref = oracle_lib.sweep(host, BETA_C, 2, 31, 12, trace=True)
    else:
        ref = oracle_lib.sweep_fmt(host, BETA_C, fmt, 2, 31, 12, trace=True)
    assert torch.equal(src, keep)
    assert np.array_equal(dst.cpu().numpy(), host)
    assert np.array_equal(me.cpu().numpy(), ref)


def test_fused_full_size_16384_crops_and_trace(dev, oracle_lib):
    # The benchmark's lattice and launch configuration: L = 16384, hot start, beta_c.
    L, n, seed = 16384, 64, 1
    _say("fused full-size", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    scratch = torch.empty_like(s)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused(s, scratch, L, BETA_C, "exact", n, seed, 0, trace)
    torch.cuda.synchronize()
    for (r0, c0, h, w) in [(0, 0, 16, 64), (L - 8, L - 40, 16, 80), (8191, 4097, 24, 24), (100, L - 1, 5, 3)]:
        ref = oracle_lib.crop(L, seed, BETA_C, n, 0, r0, c0, h, w)
        rows = [(r0 + a) % L for a in range(h)]
        cols = [(c0 + b) % L for b in range(w)]
        assert np.array_equal(s[rows][:, cols].cpu().numpy(), ref), (r0, c0)
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising_observables(s, L, out)
    assert out.tolist() == trace[-1].tolist()
    # the same run through the two-launch path: identical lattice and trace
    s2 = torch.empty_like(s)
    dev.ising_init(s2, L, seed)
    tr2 = torch.empty_like(trace)
    dev.ising_sweep(s2, L, BETA_C, n, seed, 0, tr2)
    assert torch.equal(s, s2)
    assert torch.equal(trace, tr2)


def _fused_equals_two_launch_path(dev, L, n, seed, offset, bands_opt):
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed)
    ref = s.clone()
    tr_ref = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(ref, L, BETA_C, n, seed, offset, tr_ref)
    scratch = torch.zeros_like(s)
    tr = torch.empty_like(tr_ref)
    old = dev.ising_get_option("fused_bands")
    dev.ising_set_option("fused_bands", bands_opt)
    try:
        dev.ising_sweep_fused(s, scratch, L, BETA_C, "exact", n, seed, offset, tr)
    finally:
        dev.ising_set_option("fused_bands", old)
    assert torch.equal(s, ref), (L, bands_opt)
    assert torch.equal(tr, tr_ref), (L, bands_opt)
    del s, ref, scratch
    torch.cuda.empty_cache()


def test_fused_largest_full_row_lattice_and_bands_above_it(dev):
    # L = 65536 with rows kept whole (option fused_bands = 2): 1024 threads per workgroup, 72 KiB of
    # LDS.  L = 65600 (1025 groups): above the full-row limit the two-sweep pass runs in column bands
    # whatever the option (17 bands of 60 or 61 groups, strips of 64 rows).  Both equal the in-place
    # two-launch path.
    for L, n, opt in ((65536, 2, 2), (65600, 2, 2), (65600, 2, 0)):
        _say("fused large", L, n, opt)
        _fused_equals_two_launch_path(dev, L, n, 5, 9, opt)


def test_fused_pairs_at_the_widest_rows_they_take(dev):
    # The two-sweep pass with two steps per settle up to 512 groups per row, kept as rows (option
    # fused_bands = 2): L = 32768 (512 threads per workgroup, 86 KiB of LDS, 384 strips of 84 and 86
    # rows) and L = 32704 (511 groups: one idle thread, rows loaded lane by lane); both equal the
    # in-place two-launch path over two passes
    for L, n in ((32768, 4), (32704, 4)):
        _say("fused pairs wide", L, n)
        _fused_equals_two_launch_path(dev, L, n, 8, 21, 2)


def test_fused_default_bands_above_16384(dev):
    # Above L = 16384 the two-sweep pass runs in column bands by default, with strip heights chosen
    # from the waves per SIMD: L = 16448 (257 groups: 5 bands of 51 or 52), 24576 (7 bands of 54 or
    # 55), 32768 (9 bands of 56 or 57), 49152 (13 bands of 59 or 60, 128-row strips); two passes each
    for L, n in ((16448, 4), (24576, 4), (32768, 4), (49152, 4)):
        _say("fused default bands", L, n)
        _fused_equals_two_launch_path(dev, L, n, 13, 7, 0)


def test_fused_strip_height_divides_odd_multiple_of_64(dev):
    # L = 64 * 769: the tallest two-sweep strip that leaves enough waves (128 rows) does not divide L,
    # so the strips must be 64 rows tall; every row of the lattice must still be swept
    L, n = 64 * 769, 2
    _say("fused odd multiple of 64", L)
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, 5)
    ref = base.clone()
    ref_tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fmt(ref, L, BETA_C, "exact", n, 5, 0, ref_tr)
    scratch = torch.empty_like(base)
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused(base, scratch, L, BETA_C, "exact", n, 5, 0, tr)
    assert torch.equal(base, ref)
    assert torch.equal(tr, ref_tr)
    del base, ref, scratch
    torch.cuda.empty_cache()


def test_fused_rejects_overlap(dev):
    s = torch.empty((128, 128), dtype=torch.int8, device="cuda")
    with pytest.raises(dev.IsingError):
        dev.ising_sweep_fused(s, s, 128, BETA_C, "exact", 2, 1)
    with pytest.raises(dev.IsingError):
        dev.ising_sweep_fused_step(s, s, 128, BETA_C, "exact", 1, 0)


def test_fused_steps_replay_in_a_hip_graph(dev):
    # A caller that keeps its own pair of buffers can capture alternating steps once and replay
    # them: every launch of the path is a kernel (the trace slot is cleared by a kernel, not a
    # memset).  Each replay, with eager work in between, must equal the eager sequence.
    L, n, seed = 4096, 4, 9
    a = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(a, L, seed)
    start = a.clone()
    b = torch.empty_like(a)
    me = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    # eager reference: sweeps t = 0 .. n - 1 from the same start
    ref = start.clone()
    ref_tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(ref, L, BETA_C, n, seed, 0, ref_tr)
    ref_state = start.clone()
    dev.ising_sweep(ref_state, L, BETA_C, n, seed, 0)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    a.copy_(start)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        src, dst = a, b
        for i in range(n):
            dev.ising_sweep_fused_step(src, dst, L, BETA_C, "exact", seed, i, me[i], stream=s)
            src, dst = dst, src
    # the capture recorded sweeps 0..3; replaying recomputes them from `a`
    a.copy_(start)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(a, ref_state), rep
        assert torch.equal(me, ref_tr[:n]), rep
        x = a.float().sum()                      # eager work between replays
        torch.cuda.synchronize()
        assert int(x.item()) == int(ref_state.float().sum().item())
        a.copy_(start)


def test_two_streams_at_once_match_one_at_a_time(dev):
    L, n = 4096, 6
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    lat = [torch.empty((L, L), dtype=torch.int8, device="cuda") for _ in range(2)]
    scr = [torch.empty_like(lat[0]) for _ in range(2)]
    tr = [torch.empty((n, 2), dtype=torch.int64, device="cuda") for _ in range(2)]
    for k in range(2):
        dev.ising_init(lat[k], L, 100 + k)
    torch.cuda.synchronize()
    for i in range(0, n, 2):                      # interleaved pairs of fused sweeps on two streams
        for k, st in enumerate((s1, s2)):
            dev.ising_sweep_fused(lat[k], scr[k], L, BETA_C, "exact", 2, 100 + k, i, tr[k][i:i + 2], stream=st)
    torch.cuda.synchronize()
    for k in range(2):
        ref = torch.empty_like(lat[k])
        dev.ising_init(ref, L, 100 + k)
        rt = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        dev.ising_sweep(ref, L, BETA_C, n, 100 + k, 0, rt)
        assert torch.equal(lat[k], ref), k
        assert torch.equal(tr[k], rt), k
