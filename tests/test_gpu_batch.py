"""GPU parity of the batched persistent form: many replicas of uneven L and temperature in one
launch.  Each replica must equal the oracle's single-lattice chain of its (L, beta, seed) bit for
bit (every spin and every traced (M, E)), and the FP64 moments must equal a sequential evaluation
of the trace.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))

REPLICAS = [(32, 0.5, 1001), (64, BETA_C, 1002), (192, 0.41, 1003), (128, 0.0, 1004), (320, 1 / 2.6, 1005),
            (256, math.inf, 1006), (512, BETA_C, 1007), (32, 0.3, 1008), (64, 1 / 2.2, 1009)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_11714_amd import ising
    ising.library()
    return ising


def _replica(dev, ws, n, j, L):
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_batch_unpack(ws, n, j, s)
    return s.cpu().numpy()


@pytest.mark.parametrize("slab_sites,depth", [(-1, 1), (4096, 1), (4096, 4), (16384, 2)])
def test_batch_matches_oracle(dev, oracle_lib, slab_sites, depth):
    # 9 sweeps = 18 colour updates: with 4 updates between exchanges the last period is partial
    n_therm, n_meas = 3, 6
    print("batch", len(REPLICAS), slab_sites, depth, flush=True)
    try:
        dev.ising_set_option("batch_slab_sites", slab_sites)
        dev.ising_set_option("batch_depth", depth)
        moments, trace, ws = dev.batch_run(REPLICAS, n_therm, n_meas, start=0, sweep_offset=40)
        torch.cuda.synchronize()
    finally:
        dev.ising_set_option("batch_slab_sites", 0)
        dev.ising_set_option("batch_depth", 0)
    for j, (L, beta, seed) in enumerate(REPLICAS):
        host = oracle_lib.init(L, seed)
        oracle_lib.sweep(host, beta, n_therm, seed, 40)
        ref = oracle_lib.sweep(host, beta, n_meas, seed, 40 + n_therm, trace=True)
        assert np.array_equal(_replica(dev, ws, len(REPLICAS), j, L), host), (L, beta)
        assert np.array_equal(trace[j].cpu().numpy(), ref), (L, beta)
        # FP64 moments in sweep order: the oracle's plain sums, bit for bit
        assert moments[j].cpu().tolist() == oracle_lib.moments(ref, L * L).tolist(), (L, beta)


def test_batch_equals_single_lattice_path(dev):
    reps = [(64, BETA_C, 7), (256, 0.4, 8), (512, 0.5, 9)]
    _, trace, ws = dev.batch_run(reps, 0, 5, start=0, sweep_offset=2)
    for j, (L, beta, seed) in enumerate(reps):
        p = torch.empty(L * L // 32, dtype=torch.int32, device="cuda")
        dev.ising_init_packed(p, L, seed)
        t = torch.empty((5, 2), dtype=torch.int64, device="cuda")
        dev.ising_sweep_packed(p, L, beta, 5, seed, 2, t)
        s = torch.empty((L, L), dtype=torch.int8, device="cuda")
        dev.ising_unpack(p, L, s)
        assert np.array_equal(_replica(dev, ws, len(reps), j, L), s.cpu().numpy())
        assert torch.equal(trace[j], t)


def test_batch_schedules_and_continuation_identical(dev):
    # every workgroup size with every split of the replicas into row slabs (1, 2, 4 or 8 slabs of
    # at least 16 rows) and every number of colour updates between row exchanges gives the same
    # chains
    reps = REPLICAS
    ref = None
    try:
        for sites in (-1, 65536, 16384, 4096, 1024):
            dev.ising_set_option("batch_slab_sites", sites)
            for depth, per_cu in (((1, 1),) if sites == -1 else ((1, 1), (2, 2), (4, 1), (4, 2))):
                dev.ising_set_option("batch_depth", depth)
                dev.ising_set_option("batch_lists_per_cu", per_cu)
                for threads in (256, 512, 1024):
                    print("schedule", sites, depth, per_cu, threads, flush=True)
                    dev.ising_set_option("batch_threads", threads)
                    mo, tr, ws = dev.batch_run(reps, 2, 5, start=0)
                    if ref is None:
                        ref = (mo, tr)
                    else:
                        assert torch.equal(mo, ref[0]) and torch.equal(tr, ref[1]), (sites, depth, per_cu, threads)
        for k in ("batch_threads", "batch_slab_sites", "batch_depth", "batch_lists_per_cu"):
            dev.ising_set_option(k, 0)
        mo, tr, _ = dev.batch_run(reps, 2, 5, start=0)          # autotuned schedule
        assert torch.equal(mo, ref[0]) and torch.equal(tr, ref[1])
        assert len(dev.ising_batch_schedule(reps)) == 4
        # 2 + 5 sweeps in one call == 2 therm, then continue for the 5 measured ones
        for sites, depth, threads in ((-1, 1, 512), (4096, 1, 256), (4096, 4, 512)):
            print("continuation", sites, depth, threads, flush=True)
            dev.ising_set_option("batch_slab_sites", sites)
            dev.ising_set_option("batch_depth", depth)
            dev.ising_set_option("batch_threads", threads)
            _, _, ws = dev.batch_run(reps, 2, 0, start=0)
            mo2, tr2, _ = dev.batch_run(reps, 0, 5, start=2, sweep_offset=2, workspace=ws)
            assert torch.equal(tr2, ref[1]) and torch.equal(mo2, ref[0]), (sites, depth, threads)
    finally:
        for k in ("batch_threads", "batch_slab_sites", "batch_depth", "batch_lists_per_cu"):
            dev.ising_set_option(k, 0)


def test_batch_graph_replay_deterministic(dev):
    reps = [(128, BETA_C, 5), (32, 0.6, 6)]
    ws = torch.empty(dev.ising_batch_workspace_bytes(reps), dtype=torch.uint8, device="cuda")
    out = []
    for _ in range(3):
        mo, tr, _ = dev.batch_run(reps, 4, 4, start=1, workspace=ws)
        torch.cuda.synchronize()
        out.append((mo.clone(), tr.clone()))
    for mo, tr in out[1:]:
        assert torch.equal(mo, out[0][0]) and torch.equal(tr, out[0][1])


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_batch_lowprec_matches_oracle(dev, oracle_lib, fmt):
    reps = [(32, BETA_C, 11), (128, 0.45, 12)]
    _, trace, ws = dev.batch_run(reps, 1, 4, fmt=fmt)
    for j, (L, beta, seed) in enumerate(reps):
        host = oracle_lib.init(L, seed)
        oracle_lib.sweep_fmt(host, beta, fmt, 1, seed, 0)
        ref = oracle_lib.sweep_fmt(host, beta, fmt, 4, seed, 1, trace=True)
        assert np.array_equal(_replica(dev, ws, 2, j, L), host)
        assert np.array_equal(trace[j].cpu().numpy(), ref)


def test_batch_ordered_start_below_tc(dev, oracle_lib):
    # start 3: beta > beta_c begins from all +1, the others from their hot start
    reps = [(64, 0.5, 21), (64, 0.4, 22)]
    _, trace, ws = dev.batch_run(reps, 0, 3, start=3)
    for j, (L, beta, seed) in enumerate(reps):
        host = np.ones((L, L), dtype=np.int8) if beta > BETA_C else oracle_lib.init(L, seed)
        ref = oracle_lib.sweep(host, beta, 3, seed, 0, trace=True)
        assert np.array_equal(_replica(dev, ws, 2, j, L), host)
        assert np.array_equal(trace[j].cpu().numpy(), ref)
