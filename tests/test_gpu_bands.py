"""GPU parity of the two-sweep pass in column bands (one wave per band and strip, the default above
L = 16384 and, with option "fused_bands", from L = 4096): k_sweep_fused2pb (two steps per tie settle, the
default) and k_sweep_fused2b (one step per settle, option "fused_pairs" = 0).

A band's wave recomputes one group on either side of its own groups and takes its group-edge
neighbours by a lane shift; every decision uses the site's own uniform, so the lattice and the (M, E)
trace must equal the oracle's half-sweeps bit for bit: against the oracle on full 4096^2 lattices
(two bands of 32 groups, both wrapping round the seam), against the two-launch path for every strip
height, for bands of unequal width (L = 4160: 65 groups), at 16384^2, and as the default pass at
L = 20480 and 24576 against both the two-launch path and the full-row pass.
"""
import contextlib
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


@contextlib.contextmanager
def options(dev, **kv):
    old = {k: dev.ising_get_option(k) for k in kv}
    try:
        for k, v in kv.items():
            dev.ising_set_option(k, v)
        yield
    finally:
        for k, v in old.items():
            dev.ising_set_option(k, v)


def _to_dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("pairs", [1, 0])
@pytest.mark.parametrize("L,beta,n,seed,offset,fmt", [
    (4096, BETA_C, 2, 1, 0, "exact"), (4096, 0.3, 4, 2, 7, "exact"), (4096, 0.7, 3, 3, 2**32 - 3, "exact"),
    (4096, BETA_C, 4, 4, 0, "bf16"), (4096, 0.45, 2, 5, 1, "fp16"), (4096, 0.0, 2, 6, 0, "exact"),
    (4096, math.inf, 2, 7, 0, "exact")])
def test_band_pass_matches_oracle(dev, oracle_lib, L, beta, n, seed, offset, fmt, pairs):
    # pairs: the band's walk settles two steps' tied words together (1, the default) or one step's (0)
    _say("bands vs oracle", L, beta, n, seed, offset, fmt, pairs)
    host = inputs.random_lattice(L, seed=L + n + seed)
    s, scratch = _to_dev(host), torch.empty((L, L), dtype=torch.int8, device="cuda")
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    with options(dev, fused_bands=1, fused_pairs=pairs):
        dev.ising_sweep_fused(s, scratch, L, beta, fmt, n, seed, offset, trace)
    if fmt == "exact":
        ref = oracle_lib.sweep(host, beta, n, seed, offset, trace=True)
    else:
        ref = oracle_lib.sweep_fmt(host, beta, fmt, n, seed, offset, trace=True)
    assert np.array_equal(s.cpu().numpy(), host)
    assert np.array_equal(trace.cpu().numpy(), ref)


@pytest.mark.parametrize("L", [4096, 4160, 8192])
def test_band_pass_equals_two_launch_path_for_every_strip_height(dev, L):
    n, seed = 4, 11
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, seed)
    ref = base.clone()
    ref_tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(ref, L, BETA_C, n, seed, 3, ref_tr)
    scratch = torch.empty_like(base)
    for R in (2, 4, 8, 16, 32, 64, 128, 256):
        if L % R:
            continue
        for alternate, pairs in ((1, 1), (0, 1), (1, 0), (0, 0)):
            _say("bands strip height", L, R, alternate, pairs)
            s = base.clone()
            tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
            with options(dev, fused_bands=1, band_rows=R, fused_alternate=alternate, fused_pairs=pairs):
                dev.ising_sweep_fused(s, scratch, L, BETA_C, "exact", n, seed, 3, tr)
            assert torch.equal(s, ref), (L, R, alternate, pairs)
            assert torch.equal(tr, ref_tr), (L, R, alternate, pairs)


def test_band_pair_is_two_sweeps_out_of_place(dev, oracle_lib):
    L, seed, t = 4096, 21, 40
    host = inputs.random_lattice(L, seed=5)
    src = _to_dev(host)
    keep = src.clone()
    dst = torch.empty_like(src)
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    with options(dev, fused_bands=1, xcd_remap=0):
        dev.ising_sweep_fused_pair(src, dst, L, BETA_C, "exact", seed, t, out)
    ref = oracle_lib.sweep(host, BETA_C, 2, seed, t, trace=True)
    assert torch.equal(src, keep)
    assert np.array_equal(dst.cpu().numpy(), host)
    assert out.cpu().numpy().tolist() == ref.reshape(-1).tolist()


def test_band_pass_full_size_16384(dev):
    L, n, seed = 16384, 6, 1
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, seed)
    ref = base.clone()
    ref_tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep(ref, L, BETA_C, n, seed, 0, ref_tr)
    scratch = torch.empty_like(base)
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    _say("bands 16384")
    with options(dev, fused_bands=1):
        dev.ising_sweep_fused(base, scratch, L, BETA_C, "exact", n, seed, 0, tr)
    assert torch.equal(base, ref)
    assert torch.equal(tr, ref_tr)
    del base, ref, scratch
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L,n,seed", [(20480, 5, 3), (24576, 4, 8)])
def test_default_band_pass_between_16384_and_65536(dev, L, n, seed):
    """Above L = 16384 the default two-sweep pass runs in column bands (20480: 6 bands of 53-54 groups;
    24576: 7 bands); it must equal both the two-launch path and the full-row pass (option
    "fused_bands" = 2), lattice and trace, over an odd and an even sweep count."""
    base = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(base, L, seed)
    ref = base.clone()
    ref_tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    _say("default bands", L, n, seed, "two-launch reference")
    dev.ising_sweep(ref, L, BETA_C, n, seed, 7, ref_tr)
    scratch = torch.empty_like(base)
    rows = base.clone()
    tr = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    _say("default bands", L, n, seed, "band pass")
    with options(dev, fused_bands=0):
        dev.ising_sweep_fused(base, scratch, L, BETA_C, "exact", n, seed, 7, tr)
    assert torch.equal(base, ref)
    assert torch.equal(tr, ref_tr)
    tr.zero_()
    _say("default bands", L, n, seed, "full-row pass")
    with options(dev, fused_bands=2):
        dev.ising_sweep_fused(rows, scratch, L, BETA_C, "exact", n, seed, 7, tr)
    assert torch.equal(rows, ref)
    assert torch.equal(tr, ref_tr)
    del base, ref, scratch, rows
    torch.cuda.empty_cache()
