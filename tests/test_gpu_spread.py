"""Traced sweep loops add (M, E) into spread sets of 64 cache lines and fold up to 64 launches'
sets into the trace at a time.  Runs with more traced launches than one fold takes must still give
the oracle's trace entry by entry, on every layout and path (two-sweep passes, one colour per
launch, the packed layout, rows that end in a half group), and calls on two streams at once must
give the traces of the same calls made one after the other (each call takes its own sets)."""
import math

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


def _run(dev, layout, L, beta, n, seed, offset, stream=None):
    s = torch.empty((L, L), dtype=torch.int8, device="cuda")
    dev.ising_init(s, L, seed, stream)
    tr = torch.full((n, 2), -7, dtype=torch.int64, device="cuda")
    if layout == "fused":
        scratch = torch.empty_like(s)
        dev.ising_sweep_fused(s, scratch, L, beta, "exact", n, seed, offset, tr, stream)
    elif layout == "int8":
        dev.ising_sweep(s, L, beta, n, seed, offset, tr, stream)
    else:
        planes = torch.empty(dev.ising_packed_words(L), dtype=torch.int32, device="cuda")
        dev.ising_pack(s, L, planes, stream)
        dev.ising_sweep_packed(planes, L, beta, n, seed, offset, tr, stream)
        dev.ising_unpack(planes, L, s, stream)
    return s, tr


# (layout, L, sweeps): 259 sweeps on the two-sweep path = 1 in place + 129 passes -> 128 two-sweep
# passes (two folds) and two one-sweep passes; 260 sweeps = 130 passes, folds of 64, 64 and 2; 131 sweeps of one
# colour per launch = three folds
@pytest.mark.parametrize("layout,L,n", [("fused", 128, 259), ("fused", 64, 260), ("fused", 160, 70),
                                        ("int8", 96, 131), ("packed", 128, 131), ("packed", 96, 65)])
def test_long_traces_match_oracle(dev, oracle_lib, layout, L, n):
    seed, offset = 21, 5
    print("spread", layout, L, n, flush=True)
    s, tr = _run(dev, layout, L, BETA_C, n, seed, offset)
    torch.cuda.synchronize()
    host = oracle_lib.init(L, seed)
    ref = oracle_lib.sweep(host, BETA_C, n, seed, offset, trace=True)
    assert np.array_equal(s.cpu().numpy(), host), (layout, L)
    assert np.array_equal(tr.cpu().numpy(), ref), (layout, L)


def test_two_streams_trace_independently(dev):
    L, n = 1024, 140
    print("spread two streams", L, n, flush=True)
    ref = [_run(dev, lay, L, BETA_C, n, seed, 0) for lay, seed in (("fused", 31), ("packed", 32))]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        a = _run(dev, "fused", L, BETA_C, n, 31, 0, s1)
    with torch.cuda.stream(s2):
        b = _run(dev, "packed", L, BETA_C, n, 32, 0, s2)
    torch.cuda.synchronize()
    for (rs, rt), (gs, gt) in zip(ref, (a, b)):
        assert torch.equal(rs, gs)
        assert torch.equal(rt, gt)


def test_two_host_threads_trace_independently(dev):
    # ctypes releases the GIL: two threads call into the library at once, each on its own stream, and
    # take spread sets from the shared per-device pool
    import threading
    L, n = 512, 150
    print("spread two threads", L, n, flush=True)
    jobs = [("fused", 41), ("packed", 42), ("int8", 43), ("fused", 44)]
    ref = [_run(dev, lay, L, BETA_C, n, seed, 3) for lay, seed in jobs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in jobs]
    out = [None] * len(jobs)
    errors = []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                out[i] = _run(dev, jobs[i][0], L, BETA_C, n, jobs[i][1], 3, streams[i])
            streams[i].synchronize()
        except Exception as e:  # reported below, on the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for (rs, rt), (gs, gt) in zip(ref, out):
        assert torch.equal(rs, gs)
        assert torch.equal(rt, gt)
