"""GPU parity at the largest single-GPU lattice: L = 131072 (1.7e10 spins), both layouts.

The int8 lattice (16 GiB) is swept two sweeps per pass in column bands (the benchmark's path at this
size, with a second 16 GiB buffer), the 1-bit lattice (2 GiB) by the packed kernel, and at T_c also one
colour per launch in place.  For each of T = 2.0, T_c and 2.6, 100 sweeps from
the seed-1 hot start; then a 2048 x 2048 window across the torus seam is checked against the
oracle's light-cone run (a (2048 + 4 * 100)^2 window, Sec. 3.1: after n sweeps a site depends only
on sites within distance 2n), the traced (M, E) against a fresh reduction, and the two layouts
against each other on every spin.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

L = 131072
N_SWEEPS = 100
SEED = 1
T_C = 2.0 / math.log1p(math.sqrt(2.0))


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


@pytest.mark.parametrize("T", [2.0, T_C, 2.6])
def test_largest_lattice_both_layouts(dev, oracle_lib, T):
    beta = 1.0 / T
    _say("L=131072 int8, two sweeps per pass in column bands", T)
    buf = torch.empty(2 * L * L, dtype=torch.int8, device="cuda")
    s, scratch = buf[:L * L].view(L, L), buf[L * L:].view(L, L)
    dev.ising_init(s, L, SEED)
    tr8 = torch.empty((N_SWEEPS, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused(s, scratch, L, beta, "exact", N_SWEEPS, SEED, 0, tr8)
    torch.cuda.synchronize()

    _say("L=131072 oracle window", T)
    r0, c0, h, w = L - 1024, L - 1024, 2048, 2048        # across both seams of the torus
    ref = oracle_lib.crop(L, SEED, beta, N_SWEEPS, 0, r0, c0, h, w)
    rows = torch.tensor([(r0 + a) % L for a in range(h)], device="cuda")
    cols = torch.tensor([(c0 + b) % L for b in range(w)], device="cuda")
    got = s.index_select(0, rows).index_select(1, cols).cpu().numpy()
    assert np.array_equal(got, ref)

    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising_observables(s, L, out)
    assert out.tolist() == tr8[-1].tolist()

    _say("L=131072 packed", T)
    p = torch.empty(L * L // 32, dtype=torch.int32, device="cuda")
    dev.ising_init_packed(p, L, SEED)
    trp = torch.empty((N_SWEEPS, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_packed(p, L, beta, N_SWEEPS, SEED, 0, trp)
    assert torch.equal(trp, tr8)
    dev.ising_unpack(p, L, scratch)
    assert torch.equal(scratch, s)
    del p

    if abs(T - T_C) < 1e-9:
        # and the in-place two-launch path (one colour per launch) gives the same lattice and trace
        _say("L=131072 int8 in place", T)
        dev.ising_init(scratch, L, SEED)
        tr2 = torch.empty((N_SWEEPS, 2), dtype=torch.int64, device="cuda")
        dev.ising_sweep(scratch, L, beta, N_SWEEPS, SEED, 0, tr2)
        assert torch.equal(tr2, tr8)
        assert torch.equal(scratch, s)
    del s, scratch, buf
    torch.cuda.empty_cache()
