#!/usr/bin/env python3
"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

Workload (the paper's single-lattice measurement, Sec. 4.2: time per sweep of all black and
all white sites, flips/ns = L^2 / sweep time): a periodic 16384 x 16384 int8 lattice, hot
start from seed 1, beta = beta_c = ln(1 + sqrt 2) / 2, exact-threshold acceptance, with the
(M, E) trace recorded after every sweep.  One "step" is one sweep.  The lattice is resident in
HBM before the timed region starts.

Layouts: "fused" (default) sweeps the int8 lattice two whole sweeps (both colours of each) per
pass, alternating between the lattice and a second L^2-byte buffer; "int8" runs one launch per
colour in place; "packed" is the 1-bit layout.  All three run the same chain (bit-identical spins).

With --compare (default) the line also carries the same fused workload with the acceptance test
in bfloat16 and in half ("bf16_accept", "fp16_accept": u < p with both rounded to the format, a
different chain) and the int8 and packed layouts on the exact chain.

Prints one JSON line with the throughput (spin-flip attempts per ns), the roofline of the
dominant kernel (algorithmic bytes = one read and one write of the L^2-byte lattice per launch,
over the average launch time of the timed region, from HIP events on the launch stream) and the
CPU oracle's throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BETA_C = 0.5 * math.log1p(math.sqrt(2.0))
HBM_PEAK_GBS = 8000.0
METRIC = "spin-flip attempts/ns (L=16384², T_c) + % HBM peak, exact vs bf16 accept"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1903_11714_amd", "csrc", f) for f in ("ising.hip", "philox.hpp", "rows.hpp")]
KERNEL_SOURCES_3D = KERNEL_SOURCES + [os.path.join(ROOT, "paper_1903_11714_amd", "csrc", "ising3d.hip")]


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed (string literals kept)."""
    import re
    pattern = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"', re.S)
    text = pattern.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", text)
    return " ".join(text.split())


def kernel_source_hash(sources=None) -> str:
    """Hash of the kernel sources' code (comments and layout ignored): the committed counters belong
    to the kernels while it matches."""
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_counters(layout: str, L: int) -> dict:
    """The committed rocprofv3 counter summary of this layout's kernel at this size (HBM bytes
    and VALU instructions per launch), or {} when the kernel source changed since the counters
    were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    entry = rec.get(f"{layout}_L{L}")
    sources = KERNEL_SOURCES_3D if layout.endswith("3d") else KERNEL_SOURCES
    if not entry or entry.get("source_hash") != kernel_source_hash(sources):
        return {}
    return entry


def measured_traffic(layout: str, L: int):
    """HBM bytes per launch from the committed counter summary, or None."""
    return measured_counters(layout, L).get("hbm_bytes_per_launch")


# vector ALU issue peak for 32-bit integer work: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64
# instruction takes 4 cycles on a 16-lane SIMD; integer ops have no packed two-per-lane form)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def alu_roofline(layout: str, L: int, avg_launch_ms: float):
    """Lane operations per second of the kernel's VALU instructions (count from the committed
    counters, time from this run) against the integer VALU peak, with rocprofv3's VALUBusy."""
    c = measured_counters(layout, L)
    if "valu_insts_per_launch" not in c:
        return None
    achieved = c["valu_insts_per_launch"] * 64 / (avg_launch_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
            "frac": achieved / VALU_PEAK_TOPS, "valu_busy": c.get("valu_busy_pct", 0.0) / 100.0,
            "valu_insts_per_launch": c["valu_insts_per_launch"]}


BANDS_ABOVE_L = 16384  # above this the two-sweep pass runs as column bands of one wave each

KERNEL_NAME = {
    "fused": "k_sweep_fused2p (two sweeps per launch, ties of two steps settled together)",
    "bands": "k_sweep_fused2pb (two sweeps per launch in column bands of one wave, ties of two steps settled together)",
    "int8": "k_sweep_int8 (one colour per launch)",
    "packed": "k_sweep_packed_q (one colour per launch, tie queue)",
}


def kernel_name(layout: str, L: int) -> str:
    if layout == "fused" and L > BANDS_ABOVE_L:
        return KERNEL_NAME["bands"]
    return KERNEL_NAME[layout]


FUSED_SWEEPS_PER_LAUNCH = 2

# Bytes each attempt must move at minimum for the schedule of each layout (one read and one write of
# every spin per pass): int8 with one launch per colour 4 B per sweep (read L^2 and write L^2 per
# half-sweep); int8 with both colours of a sweep in one pass 2 B (the minimum for one sweep per pass;
# the default pass makes two sweeps and so needs only 1 B, but the 2 B figure is the one a one-sweep
# schedule would be held to); 1-bit colour-split 0.375 B (both planes read, one written, per half-sweep).
BYTES_PER_ATTEMPT = {"fused": 2.0, "int8": 4.0, "packed": 0.375}


def attempts_per_launch(layout: str, L: int) -> float:
    """Site updates one launch of the layout's dominant kernel makes: two sweeps of L^2 sites for the
    two-sweep pass, one colour (L^2 / 2 sites) for the one-launch-per-colour kernels."""
    return 2.0 * L * L if layout == "fused" else 0.5 * L * L


def algorithmic_bytes(layout: str, L: int) -> float:
    """Algorithmic bytes per launch: bytes per attempt x attempts per launch."""
    return BYTES_PER_ATTEMPT[layout] * attempts_per_launch(layout, L)


def moved_bytes(layout: str, L: int) -> float:
    """Bytes one launch reads and writes when every spin moves exactly once each way: the two-sweep
    pass reads the L^2-byte lattice and writes the other buffer; the int8 half-sweep reads and writes
    the lattice; the packed half-sweep reads both colour planes (L^2 / 8) and writes one (L^2 / 16)."""
    return 3.0 * L * L / 16.0 if layout == "packed" else 2.0 * L * L


def fused_passes(n: int) -> tuple[int, int, int]:
    """(two-sweep passes, one-sweep passes, in-place sweeps) that ising_sweep_fused makes for n sweeps:
    an odd n runs its first sweep in place; the even rest goes in passes of two sweeps, an even number of
    passes in all (an odd number of two-sweep passes gives one up for two one-sweep passes)."""
    in_place = n & 1
    rest = n - in_place
    pairs = rest // 2
    if pairs & 1:
        pairs -= 1
    return pairs, rest - 2 * pairs, in_place


def copy_bandwidth(torch, L: int, stream, reps: int = 20, in_place: bool = False) -> float:
    """GB/s (bytes read + written) of a plain pass over an L^2-byte buffer: torch's device-to-device
    copy into a second buffer, or (in_place) an elementwise negation written back in place."""
    n = min(L, 16384) ** 2
    src = torch.ones(n, dtype=torch.int8, device="cuda")
    dst = src if in_place else torch.empty_like(src)

    def one():
        if in_place:
            src.neg_()
        else:
            dst.copy_(src)
    for _ in range(3):
        one()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        one()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n / (ms * 1e-3) / 1e9


CALIBRATION_MAX_BYTES = 1 << 30  # torch splits larger copies into several dispatches


def calibration_bytes(L: int) -> int:
    """Bytes of the plain copy whose counters calibrate FETCH_SIZE / WRITE_SIZE (one dispatch)."""
    return min(L * L, CALIBRATION_MAX_BYTES)


def calibration_copies(torch, nbytes: int, reps: int) -> None:
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the per-launch
    HBM traffic read from the same counters for a sweep kernel.  (int8 -> uint8 goes through an
    elementwise copy kernel that reads and writes nbytes, like a sweep; a same-dtype copy would use
    the runtime's blit kernel.)"""
    src = torch.ones(nbytes, dtype=torch.int8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


BETA_C3 = 0.2216546  # simple-cubic critical coupling (Monte Carlo estimate)


def bench_3d(ising, torch, args, stream) -> dict:
    """The cubic lattice: hot start, W warm-up sweeps, K timed sweeps with the (M, E) trace, the
    roofline of the half-sweep kernel (one read and one write of the L^3-byte lattice per launch)
    and the oracle on a bounded sample."""
    L, K, W, seed = args.L3, args.steps, args.warmup, args.seed
    beta = BETA_C3 if args.beta == BETA_C else args.beta
    dev = torch.device("cuda:0")
    lat = torch.empty((L, L, L), dtype=torch.int8, device=dev)
    ising.ising3_init(lat, L, seed, stream)
    trace = torch.empty((max(K, W, 1), 2), dtype=torch.int64, device=dev)
    if W:
        ising.ising3_sweep(lat, L, beta, W, seed, 0, trace[:W], stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    ising.ising3_sweep(lat, L, beta, K, seed, W, trace[:K], stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    launch_us = gpu_ms * 1e3 / (2 * K)
    alg = 2.0 * L ** 3
    achieved = alg / (launch_us * 1e-6) / 1e9
    cb = copy_bandwidth(torch, 16384, stream, in_place=True)  # the 3-D sweep writes back in place
    res = {
        "form": "3d",
        "metric": f"spin-flip attempts/ns (3-D, L={L}^3, beta={beta:g})",
        "value": float(L) ** 3 * K / (wall * 1e9),
        "unit": "attempts/ns",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True, "dtype": "int8", "data": "synthetic: Philox hot start from the seed (no dataset)",
        "config": {"workload": f"single periodic {L}^3 cubic lattice, beta={beta:g}, hot start seed {seed}, plain "
                               f"exact-threshold checkerboard Metropolis, int8 ({L ** 3 / 2 ** 20:.0f} MiB), one "
                               "launch per colour, (M,E) traced every sweep", "L": L, "beta": beta},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("int8_3d", L),
                     "kernel": "k_sweep3 (one colour per launch, two planes per exchange)",
                     "avg_launch_us": launch_us, "alg_bytes_per_launch": alg, "copy_GBs": cb,
                     "copy_kind": "in place", "frac_of_copy": achieved / cb if cb else None},
        "final_ME": trace[K - 1].tolist() if K else None,
    }
    del lat
    if args.compare:
        # the same chain on the 1-bit layout (bit-identical spins), for reference
        planes = torch.empty(L ** 3 // 32, dtype=torch.int32, device=dev)
        ising.ising3_init_packed(planes, L, seed, stream)
        kp = max(K // 4, 1)
        if W:
            ising.ising3_sweep_packed(planes, L, beta, W, seed, 0, trace[:W], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        ising.ising3_sweep_packed(planes, L, beta, kp, seed, W, trace[:kp], stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        res["packed_layout"] = {"value": float(L) ** 3 * kp / (pw * 1e9), "unit": "attempts/ns", "steps": kp,
                                "kernel": "k_sweep3_packed_q (one colour per launch, tie queue)",
                                "avg_launch_us": ev0.elapsed_time(ev1) * 1e3 / (2 * kp)}
        del planes
        # the same chain with both colours per pass, out of place (bit-identical spins)
        kf = max(K // 4, 2) // 2 * 2
        buf = torch.empty(2 * L ** 3, dtype=torch.int8, device=dev)
        lat, scr = buf[:L ** 3].view(L, L, L), buf[L ** 3:].view(L, L, L)
        ising.ising3_init(lat, L, seed, stream)
        if W:
            ising.ising3_sweep_fused(lat, scr, L, beta, W - W % 2, seed, 0, None, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        ising.ising3_sweep_fused(lat, scr, L, beta, kf, seed, W - W % 2, trace[:kf], stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        fw = time.perf_counter() - t0
        fl_us = ev0.elapsed_time(ev1) * 1e3 / kf
        res["fused_layout"] = {"value": float(L) ** 3 * kf / (fw * 1e9), "unit": "attempts/ns", "steps": kf,
                               "kernel": "k_sweep3_fusedq (both colours per launch, tie queue)", "avg_launch_us": fl_us,
                               "hbm_GBs": 2.0 * L ** 3 / (fl_us * 1e-6) / 1e9}
        del buf, lat, scr
    if args.copy_calibration:
        calibration_copies(torch, 16384 * 16384, args.copy_calibration)
    if not args.no_cpu_baseline:
        import oracle
        Lc = min(L, 256)
        spins = oracle.init3(Lc, seed)
        n = 16 * args.cpu_sweeps
        t0 = time.perf_counter()
        oracle.sweep3(spins, beta, n, seed, 0)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": Lc ** 3 * n / (dt * 1e9), "unit": "attempts/ns", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{n} sweeps of a {Lc}^3 lattice from the seed-{seed} hot "
                                                           f"start ({dt:.1f} s; plain C oracle, OpenMP over rows)"}
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(L: int, beta: float, seed: int, sweeps: int, one_core_L: int = 8192, one_core_sweeps: int = 2):
    """The oracle, built -O3 -march=native on this host, timed on `sweeps` sweeps of the lattice (at most
    16384^2) with every OpenMP thread, and on `one_core_sweeps` sweeps of a one_core_L^2 lattice with
    one thread; each sample is 10-20 s of host time."""
    import tempfile

    import oracle
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    flags = oracle.load_native(tmp)
    L = min(L, 16384)
    threads = oracle.num_threads()
    spins = oracle.init(L, seed)
    t0 = time.perf_counter()
    oracle.sweep(spins, beta, sweeps, seed, 0)
    dt = time.perf_counter() - t0
    del spins
    oracle.set_num_threads(1)
    Lc = min(L, one_core_L)
    spins = oracle.init(Lc, seed)
    t0 = time.perf_counter()
    oracle.sweep(spins, beta, one_core_sweeps, seed, 0)
    dt1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    return {
        "value": L * L * sweeps / (dt * 1e9),
        "unit": "attempts/ns",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{sweeps} sweeps of the full {L}x{L} lattice at beta={beta:.6g} from the seed-{seed} hot start "
                  f"({dt:.1f} s; plain C oracle, {flags}, OpenMP over the rows of each half-sweep, {threads} threads)",
        "one_core": {"value": Lc * Lc * one_core_sweeps / (dt1 * 1e9), "unit": "attempts/ns", "cores": 1,
                     "sample": f"{one_core_sweeps} sweeps of a {Lc}x{Lc} lattice, same start and beta ({dt1:.1f} s)"},
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
        "build": flags,
    }


WARM_FLOOR_S = 0.3   # GPU seconds of sweeps before anything is timed, whatever --warmup asks


def run_layout(ising, torch, layout, L, beta, seed, K, W, kernel_sweeps, stream, fmt="exact", repeats=5,
               warm_floor=WARM_FLOOR_S):
    """Hot start; W warm-up sweeps and more until `warm_floor` seconds of GPU time have gone into
    sweeps; then `repeats` timed runs of exactly K sweeps with the (M, E) trace, each bracketed by a
    device synchronisation and by events on the launch stream; then `kernel_sweeps` sweeps with every
    launch bracketed by events (one launch per two sweeps for "fused", per colour otherwise).  `fmt`
    is the acceptance format (exact, bf16 or fp16; the fused layout only)."""
    assert fmt == "exact" or layout == "fused"
    dev = torch.device("cuda:0")
    if layout in ("int8", "fused"):
        # the fused sweep's two buffers come from one allocation (their relative placement in
        # HBM is then the same on every run)
        buf = torch.empty((2 if layout == "fused" else 1) * L * L, dtype=torch.int8, device=dev)
        lat = buf[:L * L].view(L, L)
        ising.ising_init(lat, L, seed, stream)
        if layout == "fused":
            scratch = buf[L * L:].view(L, L)

            def sweep(lat, L, beta, n, seed, off, trace, st):
                ising.ising_sweep_fused(lat, scratch, L, beta, fmt, n, seed, off, trace, st)
        else:
            sweep = ising.ising_sweep
    else:
        lat = torch.empty(L * L // 32, dtype=torch.int32, device=dev)
        ising.ising_init_packed(lat, L, seed, stream)
        sweep = ising.ising_sweep_packed
    trace = torch.empty((max(K, W, 1), 2), dtype=torch.int64, device=dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def run(n, off, tr):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        sweep(lat, L, beta, n, seed, off, tr, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev0.elapsed_time(ev1)

    t = 0
    warm_ms, warm_n = 0.0, 0
    if W:
        warm_ms += run(W, t, trace[:W])[1]
        t += W
        warm_n += W
    chunk = max(K, 2)
    while warm_ms < warm_floor * 1e3 and warm_n < 100000:
        warm_ms += run(chunk, t, trace[:chunk])[1]
        t += chunk
        warm_n += chunk
    print(f"bench: {layout} ({fmt}) L={L} warm-up {warm_n} sweeps, {warm_ms:.0f} ms of GPU time", file=sys.stderr,
          flush=True)
    walls, gpus = [], []
    for _ in range(repeats):
        w, g = run(K, t, trace[:K])
        t += K
        walls.append(w)
        gpus.append(g)
    wall = statistics.median(walls)
    gpu_ms = statistics.median(gpus)
    print(f"bench: {layout} timed {repeats} x {K} sweeps: median {wall * 1e3:.3f} ms wall, {gpu_ms:.3f} ms events",
          file=sys.stderr, flush=True)
    final_ME = trace[K - 1].tolist() if K else None

    # the dominant kernel launch by launch, each bracketed by events on the launch stream (untraced)
    nk = kernel_sweeps + (kernel_sweeps & 1)
    if layout == "fused":
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nk // 2 + 1)]
        evs[0].record(stream)
        src, dst = lat, scratch
        for i in range(nk // 2):
            ising.ising_sweep_fused_pair(src, dst, L, beta, fmt, seed, t + 2 * i, None, stream)
            evs[i + 1].record(stream)
            src, dst = dst, src
    else:
        half = ising.ising_half_sweep if layout == "int8" else ising.ising_half_sweep_packed
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nk + 1)]
        evs[0].record(stream)
        for i in range(nk):
            half(lat, L, beta, seed, t + i, 1, stream)
            evs[2 * i + 1].record(stream)
            half(lat, L, beta, seed, t + i, 0, stream)
            evs[2 * i + 2].record(stream)
    torch.cuda.synchronize()
    durs = [evs[k].elapsed_time(evs[k + 1]) for k in range(len(evs) - 1)]
    del lat
    if layout == "fused":
        pairs, singles, in_place = fused_passes(K)
        # the timed region holds only two-sweep passes when K % 4 == 0 (and the trace's zeroing and one
        # fold of the spread sets per 64 passes, 4-5 us each)
        launches = pairs if (singles == 0 and in_place == 0) else 0
    else:
        launches = 2 * K
    return {
        "value": float(L) * L * K / (wall * 1e9),
        "wall_s": wall,
        "gpu_ms": gpu_ms,
        "repeats": [float(L) * L * K / (w * 1e9) for w in walls],
        "warmup_sweeps": warm_n,
        # the timed region's launches (with the traced (M, E) reduction): events on the launch
        # stream around the whole region, divided by the number of sweep launches in it
        "avg_launch_ms": gpu_ms / launches if launches else sum(durs) / len(durs),
        "avg_launch_from": "timed region" if launches else "untraced launches (K not a multiple of 4)",
        # launch by launch, without the trace
        "untraced_launch_ms": sum(durs) / len(durs),
        "final_ME": final_ME,
    }


def roofline(layout: str, L: int, avg_launch_ms: float, untraced_launch_ms: float, copy_gbs: float) -> dict:
    """HBM roofline of the dominant kernel at the algorithmic bytes per launch (bytes per attempt x
    attempts per launch), with the measured HBM traffic (committed counters, while the kernel source
    is unchanged), the bytes a pass moves when every spin goes once each way, and the vector-ALU
    roofline beside it."""
    alg = algorithmic_bytes(layout, L)
    sec = avg_launch_ms * 1e-3
    achieved = alg / sec / 1e9
    traffic = measured_traffic(layout, L)
    moved = moved_bytes(layout, L)
    roof = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": kernel_name(layout, L), "avg_launch_us": avg_launch_ms * 1e3,
        "untraced_launch_us": untraced_launch_ms * 1e3,
        "bytes_per_attempt": BYTES_PER_ATTEMPT[layout], "attempts_per_launch": attempts_per_launch(layout, L),
        "alg_bytes_per_launch": alg,
        "moved": {"bytes_per_launch": moved, "achieved": moved / sec / 1e9, "frac": moved / sec / 1e9 / HBM_PEAK_GBS},
        "measured_traffic": None if traffic is None else
        {"achieved": traffic / sec / 1e9, "frac": traffic / sec / 1e9 / HBM_PEAK_GBS},
        "alu": alu_roofline(layout, L, avg_launch_ms),
        "copy_GBs": copy_gbs,
        "copy_kind": "out of place" if layout == "fused" else "in place",
        "moved_frac_of_copy": (moved / sec / 1e9) / copy_gbs if copy_gbs else None,
    }
    return roof


COUNTER_KEYS = {
    "FETCH_SIZE": "fetch_kib_raw", "WRITE_SIZE": "write_kib_raw", "VALUBusy": "valu_busy_pct",
    "SQ_INSTS_VALU": "valu_insts_per_launch", "SQ_INSTS_SALU": "salu_insts_per_launch",
    "SQ_INSTS_LDS": "lds_insts_per_launch", "SQ_WAVES": "waves_per_launch", "SQ_WAVE_CYCLES": "wave_cycles",
    "SQ_WAIT_ANY": "wait_any_cycles", "SQ_WAIT_INST_ANY": "wait_inst_any_cycles",
    "SQ_ACTIVE_INST_ANY": "active_inst_any_cycles", "SQ_ACTIVE_INST_VALU": "active_inst_valu_cycles",
    "SQ_ACTIVE_INST_LDS": "active_inst_lds_cycles",
}
COPY_KERNEL = "direct_copy_kernel"  # the elementwise int8 -> uint8 copy of calibration_copies


def read_counters(dirs) -> dict:
    """Per-dispatch counter values from rocprofv3 --pmc CSV output: {kernel name: {counter: [value per
    dispatch]}} (a counter's rows of one dispatch are summed)."""
    import csv
    import glob
    per = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            acc = {}
            with open(f, newline="") as fh:
                for row in csv.DictReader(fh):
                    key = (row["Dispatch_Id"], row["Kernel_Name"], row["Counter_Name"])
                    acc[key] = acc.get(key, 0.0) + float(row["Counter_Value"])
            for (_, kname, cname), v in acc.items():
                per.setdefault(kname, {}).setdefault(cname, []).append(v)
    return per


def ingest_counters(key: str, layout: str, L: int, dirs, traced: str, untraced: str | None, copy_bytes: int,
                    command: str, alg_bytes: float | None = None) -> dict:
    """Write profiles/traffic.json[key] from rocprofv3 --pmc runs of this repository's bench (`dirs`):
    per-dispatch means of the kernel whose name contains `traced` (and of `untraced`, if given), the
    HBM bytes per launch with FETCH_SIZE and WRITE_SIZE each scaled by what the same counter reads for
    the plain copy of `copy_bytes` bytes each way (--copy-calibration), and the kernel source hash."""
    per = read_counters(dirs)

    def means(sub):
        names = [k for k in per if sub in k]
        if not names:
            raise SystemExit(f"bench.py: no dispatch of a kernel matching {sub!r} in {dirs}")
        out = {}
        for cname, field in COUNTER_KEYS.items():
            vals = [v for k in names for v in per[k].get(cname, [])]
            if vals:
                out[field] = sum(vals) / len(vals)
        return out, names

    entry, names = means(traced)
    entry = {"kernel": names, **entry}
    if untraced:
        u, unames = means(untraced)
        entry.update({"untraced_kernel": unames, **{f"untraced_{k}": v for k, v in u.items()}})
    copy = [k for k in per if COPY_KERNEL in k]
    if "fetch_kib_raw" in entry and "write_kib_raw" in entry and copy:
        cf = [v for k in copy for v in per[k].get("FETCH_SIZE", [])]
        cw = [v for k in copy for v in per[k].get("WRITE_SIZE", [])]
        kib = copy_bytes / 1024.0
        entry["fetch_scale"] = kib / (sum(cf) / len(cf))
        entry["write_scale"] = kib / (sum(cw) / len(cw))
        entry["copy_fetch_kib_raw"] = sum(cf) / len(cf)
        entry["copy_write_kib_raw"] = sum(cw) / len(cw)
        entry["hbm_bytes_per_launch"] = round(1024.0 * (entry["fetch_kib_raw"] * entry["fetch_scale"] +
                                                        entry["write_kib_raw"] * entry["write_scale"]))
    entry["alg_bytes_per_launch"] = algorithmic_bytes(layout, L) if alg_bytes is None else alg_bytes
    entry["source_hash"] = kernel_source_hash(KERNEL_SOURCES_3D if layout.endswith("3d") or key.startswith("int8_3d")
                                              else None)
    entry["command"] = command
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec[key] = entry
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return entry


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed sweeps per repeat")
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed sweeps first (more follow until %.1f s of GPU time has gone into sweeps)" % WARM_FLOOR_S)
    ap.add_argument("--repeats", type=int, default=5, help="timed runs of --steps sweeps; the median is reported")
    ap.add_argument("--warm-floor", type=float, default=WARM_FLOOR_S,
                    help="GPU seconds of sweeps before anything is timed (0 under a counter-collecting profiler)")
    ap.add_argument("--L", type=int, default=16384)
    ap.add_argument("--beta", type=float, default=BETA_C)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--kernel-sweeps", type=int, default=50, help="sweeps timed launch by launch")
    ap.add_argument("--cpu-sweeps", type=int, default=8, help="sweeps in the CPU-oracle sample (all threads)")
    ap.add_argument("--layout", choices=["fused", "int8", "packed"], default="fused",
                    help="fused: int8, both colours per launch, two buffers (default); int8: one launch "
                         "per colour, in place; packed: 1-bit spins, one launch per colour")
    ap.add_argument("--compare", type=int, default=1,
                    help="with the fused layout, also time the other formats and layouts on the same workload")
    ap.add_argument("--largest", type=int, default=1,
                    help="with the fused layout, also time the largest lattice (L = 131072, 100-sweep workload) on "
                         "both layouts at T = 2.0, T_c and 2.6")
    ap.add_argument("--form", choices=["plain", "precision", "batch", "3d"], default="plain",
                    help="plain: the timed sweep (default); precision: bfloat16/half vs exact chains on "
                         "the --L lattice; batch: the 255-replica Binder-crossing run in one launch; "
                         "3d: the cubic lattice (--L3, default 1024) at the 3-D critical coupling")
    ap.add_argument("--L3", type=int, default=1024, help="edge of the cubic lattice for --form 3d")
    ap.add_argument("--meas", type=int, default=None, help="measurement sweeps of the precision/batch forms")
    ap.add_argument("--therm", type=int, default=None, help="thermalisation sweeps of the precision/batch forms")
    ap.add_argument("--seeds", type=int, default=8, help="seeds per temperature and format (precision form)")
    ap.add_argument("--record", default=None,
                    help="precision/batch forms: write the full JSON record to this path and a markdown "
                         "table beside it (.md)")
    ap.add_argument("--option", action="append", default=[], metavar="NAME=VALUE",
                    help="library launch option (ising_set_option) for this run; every setting gives the same chain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run this many plain device copies of min(L^2, 2^30) bytes (counter calibration)")
    ap.add_argument("--ingest-counters", nargs="+", metavar="DIR", default=None,
                    help="no GPU run: summarise the rocprofv3 --pmc output directories DIR... of this bench "
                         "(--layout, --L, with --copy-calibration) into profiles/traffic.json")
    ap.add_argument("--traced-kernel", default=None, help="--ingest-counters: name substring of the traced kernel")
    ap.add_argument("--untraced-kernel", default=None, help="--ingest-counters: name substring of its untraced form")
    ap.add_argument("--counters-command", default="", help="--ingest-counters: the profiling commands, for the record")
    args = ap.parse_args()

    if args.ingest_counters:
        if args.form == "3d":  # one colour of the cubic lattice per launch: its L^3 bytes read and written once
            key, alg = f"int8_3d_L{args.L3}", 2.0 * args.L3 ** 3
        else:
            key, alg = f"{args.layout}_L{args.L}", None
        entry = ingest_counters(key, args.layout, args.L, args.ingest_counters, args.traced_kernel,
                                args.untraced_kernel, calibration_bytes(16384 if args.form == "3d" else args.L),
                                args.counters_command, alg)
        print(json.dumps({key: entry}))
        return 0

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(one periodic lattice per GPU, no sharding).", file=sys.stderr)
        return 2
    if args.steps < 1 or args.repeats < 1:
        print("bench.py: --steps and --repeats must be positive", file=sys.stderr)
        return 2

    import torch
    from paper_1903_11714_amd import ising

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    L, beta, seed, K, W = args.L, args.beta, args.seed, args.steps, args.warmup
    for opt in args.option:
        name, value = opt.split("=", 1)
        ising.ising_set_option(name, int(value))
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.form == "3d":
        print(json.dumps(bench_3d(ising, torch, args, stream)), flush=True)
        return 0
    if args.form != "plain":
        from paper_1903_11714_amd import studies

        def log(msg):
            print("bench: " + msg, file=sys.stderr, flush=True)
        if args.form == "precision":
            res = studies.precision_study(L=L, n_therm=args.therm if args.therm is not None else 1000,
                                          n_meas=args.meas if args.meas is not None else 10000,
                                          seeds=tuple(range(seed, seed + args.seeds)), log=log)
            table = studies.precision_table(res)
        else:
            res = studies.batch_study(n_therm=args.therm if args.therm is not None else 2000,
                                      n_meas=args.meas if args.meas is not None else 20000)
            table = studies.batch_table(res)
        res = {"form": args.form, "command": "python bench.py " + " ".join(sys.argv[1:]), **res}
        if args.record:
            os.makedirs(os.path.dirname(os.path.abspath(args.record)), exist_ok=True)
            with open(args.record, "w") as f:
                json.dump(res, f, indent=1)
            with open(os.path.splitext(args.record)[0] + ".md", "w") as f:
                f.write(f"Command: `{res['command']}`\n\n{table}\n")
        print(table, file=sys.stderr, flush=True)
        print(json.dumps({k: v for k, v in res.items() if k not in ("runs", "curves")}), flush=True)
        return 0

    main = run_layout(ising, torch, args.layout, L, beta, seed, K, W, args.kernel_sweeps, stream,
                      repeats=args.repeats, warm_floor=args.warm_floor)
    lat_bytes = L * L // 8 if args.layout == "packed" else L * L
    layout_text = {
        "fused": f"int8 layout, two sweeps per launch, lattice + scratch buffer ({2 * lat_bytes / 2**20:.0f} MiB)",
        "int8": f"int8 layout, one launch per colour, in place ({lat_bytes / 2**20:.0f} MiB)",
        "packed": f"1-bit layout, one launch per colour ({lat_bytes / 2**20:.0f} MiB)",
    }[args.layout]
    # context for the roofline: a plain pass over an L^2-byte buffer on the same GPU (out of place, as
    # the fused sweep moves its bytes; in place for the one-launch-per-colour kernels)
    cb = copy_bandwidth(torch, L, stream, in_place=args.layout != "fused")
    result = {
        "metric": METRIC,
        "value": main["value"],
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": main["wall_s"] * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 (1-bit spins)" if args.layout == "packed" else "int8",
        "data": "synthetic: Philox hot start from the seed (no dataset)",
        "config": {
            "workload": f"single periodic {L}x{L} lattice, beta={beta:.6g}"
                        f"{' (T_c)' if abs(beta - BETA_C) < 1e-12 else ''}, hot start seed {seed}, plain "
                        f"exact-threshold checkerboard Metropolis, {layout_text}, (M,E) traced every sweep",
            "L": L, "beta": beta, "layout": args.layout, "sweeps_timed": K,
        },
        "timing": {"repeats": args.repeats, "per_repeat_attempts_per_ns": main["repeats"],
                   "statistic": "median of the repeats", "warmup_sweeps_run": main["warmup_sweeps"],
                   "warmup_floor_gpu_s": WARM_FLOOR_S, "avg_launch_from": main["avg_launch_from"]},
        "roofline": roofline(args.layout, L, main["avg_launch_ms"], main["untraced_launch_ms"], cb),
        "gpu_event_ms": main["gpu_ms"],
        "final_ME": main["final_ME"],
    }
    if args.compare and args.layout == "fused":
        # the same workload with the acceptance test in bfloat16 and in half (the chain differs:
        # u < p with both rounded to the format), on the same fused kernel
        for fmt in ("bf16", "fp16"):
            low = run_layout(ising, torch, "fused", L, beta, seed, K, W, args.kernel_sweeps, stream, fmt=fmt,
                             repeats=3, warm_floor=args.warm_floor)
            r = roofline("fused", L, low["avg_launch_ms"], low["untraced_launch_ms"], cb)
            result[f"{fmt}_accept"] = {
                "value": low["value"], "unit": "attempts/ns", "steps": K, "kernel": KERNEL_NAME["fused"],
                "avg_launch_us": low["avg_launch_ms"] * 1e3, "hbm_GBs": r["achieved"], "hbm_frac": r["frac"],
                "vs_exact": low["value"] / main["value"], "final_ME": low["final_ME"],
            }
        # the same workload on the other layouts (same chain, bit-identical spins), for reference
        ks = max(K // 4, 1)
        for lay in ("int8", "packed"):
            other = run_layout(ising, torch, lay, L, beta, seed, ks, W, args.kernel_sweeps, stream, repeats=3,
                               warm_floor=args.warm_floor)
            r = roofline(lay, L, other["avg_launch_ms"], other["untraced_launch_ms"], 0.0)
            result[f"{lay}_layout"] = {
                "value": other["value"], "unit": "attempts/ns", "steps": ks, "kernel": KERNEL_NAME[lay],
                "avg_launch_us": other["avg_launch_ms"] * 1e3, "hbm_GBs": r["achieved"], "hbm_frac": r["frac"],
                "bytes_per_attempt": BYTES_PER_ATTEMPT[lay],
            }
    if args.largest and args.layout == "fused" and L != LARGEST_L:
        result["largest"] = bench_largest(ising, torch, stream, seed, warm_floor=args.warm_floor)
    if args.copy_calibration:
        calibration_copies(torch, calibration_bytes(L), args.copy_calibration)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(L, beta, seed, args.cpu_sweeps)
    print(json.dumps(result), flush=True)
    return 0


LARGEST_L = 131072


def bench_largest(ising, torch, stream, seed: int, temps=(2.0, 1.0 / BETA_C, 2.6), K: int = 8,
                  warm_floor: float = WARM_FLOOR_S) -> dict:
    """The largest single-GPU lattice (L = 131072: 16 GiB int8, 2 GiB 1-bit), hot start, at three
    temperatures on both layouts: throughput over 3 x K timed sweeps (after the warm-up floor) and the
    roofline of each layout's dominant kernel."""
    out = {"L": LARGEST_L, "sweeps_timed": K, "runs": []}
    layouts = ("fused", "packed")
    for T in temps:
        for lay in layouts:
            r = run_layout(ising, torch, lay, LARGEST_L, 1.0 / T, seed, K, 0, 4, stream, repeats=3,
                           warm_floor=warm_floor)
            roof = roofline(lay, LARGEST_L, r["avg_launch_ms"], r["untraced_launch_ms"], 0.0)
            out["runs"].append({"T": T, "layout": lay, "value": r["value"], "unit": "attempts/ns",
                                "per_repeat": r["repeats"], "kernel": kernel_name(lay, LARGEST_L),
                                "avg_launch_us": roof["avg_launch_us"], "hbm_GBs": roof["achieved"],
                                "hbm_frac": roof["frac"], "bytes_per_attempt": roof["bytes_per_attempt"],
                                "moved_frac": roof["moved"]["frac"], "final_ME": r["final_ME"]})
            torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    sys.exit(main())
