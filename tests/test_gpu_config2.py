"""The benchmark's workload end to end: a 16384^2 lattice, hot start from seed 1, beta_c, 1000
sweeps through the benchmark's path (two sweeps per pass over the lattice, alternating with a
second buffer).

The oracle's 2048^2 light-cone block of this run, across both torus seams, is pinned in
tests/golden/config2_window_L16384_n1000.json (written by tests/golden/make_config2_window.py,
which calls only the oracle): the GPU block must hash to the same SHA-256.  The same 1000 sweeps
through the two-launch path must give the identical lattice and (M, E) trace.
"""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_window_L16384_n1000.json")


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


def test_benchmark_run_matches_the_oracle_window_after_1000_sweeps(dev):
    with open(GOLDEN) as f:
        rec = json.load(f)
    L, seed, n, off = rec["L"], rec["seed"], rec["n_sweeps"], rec["sweep_offset"]
    beta = 0.5 * math.log1p(math.sqrt(2.0))
    assert beta == rec["beta"]
    _say("config 2 run", L, n)
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    scratch = torch.empty_like(s)
    dev.ising_init(s, L, seed)
    trace = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    dev.ising_sweep_fused(s, scratch, L, beta, "exact", n, seed, off, trace)
    torch.cuda.synchronize()
    rows = torch.tensor([(rec["r0"] + a) % L for a in range(rec["h"])], device="cuda")
    cols = torch.tensor([(rec["c0"] + b) % L for b in range(rec["w"])], device="cuda")
    block = np.ascontiguousarray(s.index_select(0, rows).index_select(1, cols).cpu().numpy())
    assert int(block.astype(np.int64).sum()) == rec["sum"]
    assert int(block[0].astype(np.int64).sum()) == rec["first_row_sum"]
    assert int(block[:, 0].astype(np.int64).sum()) == rec["first_col_sum"]
    assert hashlib.sha256(block.tobytes()).hexdigest() == rec["sha256_int8_row_major"]
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    dev.ising_observables(s, L, out)
    assert out.tolist() == trace[-1].tolist()
    _say("config 2 run, two-launch path")
    s2 = torch.empty_like(s)
    dev.ising_init(s2, L, seed)
    tr2 = torch.empty_like(trace)
    dev.ising_sweep(s2, L, beta, n, seed, off, tr2)
    assert torch.equal(s, s2)
    assert torch.equal(trace, tr2)
    del s, s2, scratch
    torch.cuda.empty_cache()
