"""The entry point that allocates nothing (ising_sweep_fused_static): its second lattice buffer is the
library's static device array.  Two calls in a row, the second on a smaller lattice, must give the
lattice and (M, E) trace of ising_sweep_fused with a caller-owned scratch buffer, bit for bit."""
import math
import sys

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


def test_static_scratch_matches_caller_scratch_on_two_calls(dev):
    for L, n, seed, fmt in ((8192, 6, 3, "exact"), (4096, 5, 4, "bf16"), (192, 7, 5, "exact")):
        print("no-alloc", L, n, seed, fmt, flush=True)
        sys.stdout.flush()
        a = torch.empty((L, L), dtype=torch.int8, device="cuda")
        dev.ising_init(a, L, seed)
        b = a.clone()
        scratch = torch.empty_like(a)
        ta = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        tb = torch.empty_like(ta)
        dev.ising_sweep_fused(a, scratch, L, BETA_C, fmt, n, seed, 11, ta)
        dev.ising_sweep_fused_static(b, L, BETA_C, fmt, n, seed, 11, tb)
        torch.cuda.synchronize()
        assert torch.equal(a, b), L
        assert torch.equal(ta, tb), L


def test_static_scratch_rejects_lattices_past_its_size(dev):
    L = 8256                                    # L^2 > 64 MiB (the lattice part of the array)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    with pytest.raises(dev.IsingError):
        dev.ising_sweep_fused_static(s, L, BETA_C, "exact", 2, 1, 0)


def test_static_spread_sets_over_several_folds(dev):
    # the traced launches' spread sets sit in the static array too: more traced launches than one
    # fold takes (64), on the two-sweep path (L = 192) and in place (L = 160, a half group per row)
    for L, n, seed in ((192, 261, 6), (160, 70, 7)):
        print("no-alloc long trace", L, n, seed, flush=True)
        a = torch.empty((L, L), dtype=torch.int8, device="cuda")
        dev.ising_init(a, L, seed)
        b = a.clone()
        scratch = torch.empty_like(a)
        ta = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        tb = torch.full_like(ta, -3)
        dev.ising_sweep_fused(a, scratch, L, BETA_C, "exact", n, seed, 2, ta)
        dev.ising_sweep_fused_static(b, L, BETA_C, "exact", n, seed, 2, tb)
        torch.cuda.synchronize()
        assert torch.equal(a, b), L
        assert torch.equal(ta, tb), L
