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


def kernel_source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
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


FUSED_MAX_L = 65536  # one workgroup thread per 64-column group, at most 1024 threads

KERNEL_NAME = {
    "fused": "k_sweep_fused2q (two sweeps per launch, tie queue)",
    "int8": "k_sweep_int8 (one colour per launch)",
    "packed": "k_sweep_packed_q (one colour per launch, tie queue)",
}


FUSED_SWEEPS_PER_LAUNCH = 2


def algorithmic_bytes(layout: str, L: int) -> float:
    """Bytes one launch must move: fused reads the L^2-byte lattice and writes the other buffer
    (for its two sweeps); int8 reads and writes the lattice for one colour; packed reads both
    colour planes (L^2 / 8 bytes) and writes one (L^2 / 16 bytes)."""
    return 3.0 * L * L / 16.0 if layout == "packed" else 2.0 * L * L


def fused_launches(n: int) -> int:
    """Passes ising_sweep_fused makes for an even count n: two sweeps each, in an even number of
    passes (an odd number of two-sweep passes gives one up for two one-sweep passes)."""
    pairs = n // 2
    if pairs % 2:
        pairs -= 1
    return pairs + (n - 2 * pairs)


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


def cpu_baseline(L: int, beta: float, seed: int, sweeps: int):
    """The oracle on `sweeps` sweeps of the same lattice (at most 16384^2, so the sample stays
    around ten seconds of host time)."""
    import oracle
    L = min(L, 16384)
    spins = oracle.init(L, seed)
    t0 = time.perf_counter()
    oracle.sweep(spins, beta, sweeps, seed, 0)
    dt = time.perf_counter() - t0
    return {
        "value": L * L * sweeps / (dt * 1e9),
        "unit": "attempts/ns",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{sweeps} sweeps of the full {L}x{L} lattice at T_c from the seed-{seed} hot start "
                  f"({dt:.1f} s; plain C oracle, OpenMP over the rows of each half-sweep)",
    }


def run_layout(ising, torch, layout, L, beta, seed, K, W, kernel_sweeps, stream, fmt="exact"):
    """Hot start, W warm-up sweeps, K timed sweeps with the (M, E) trace, then `kernel_sweeps`
    sweeps with every launch bracketed by events (one launch per two sweeps for "fused", per
    colour otherwise).  `fmt` is the acceptance format of the fused layout (exact, bf16 or fp16)."""
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
    warm_trace = torch.empty((max(W, 1), 2), dtype=torch.int64, device=dev)
    trace = torch.empty((max(K, 1), 2), dtype=torch.int64, device=dev)
    if W:
        sweep(lat, L, beta, W, seed, 0, warm_trace[:W], stream)
    torch.cuda.synchronize()
    print(f"bench: {layout} ({fmt}) L={L} warmup={W} done", file=sys.stderr, flush=True)

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sweep(lat, L, beta, K, seed, W, trace[:K], stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    print(f"bench: {layout} timed {K} sweeps in {wall:.3f} s wall, {gpu_ms:.1f} ms events", file=sys.stderr,
          flush=True)
    final_ME = trace[K - 1].tolist() if K else None

    # dominant kernel: each launch bracketed by events on the launch stream
    nk = kernel_sweeps + (kernel_sweeps & 1)
    t = W + K
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
    launches = fused_launches(K) if layout == "fused" else 2 * K
    return {
        "value": float(L) * L * K / (wall * 1e9),
        "wall_s": wall,
        "gpu_ms": gpu_ms,
        # the timed region's launches (with the traced (M, E) reduction): events on the launch
        # stream around the whole region, divided by the number of sweep launches in it
        "avg_launch_ms": gpu_ms / launches if launches else float("nan"),
        # launch by launch, without the trace
        "untraced_launch_ms": sum(durs) / len(durs),
        "final_ME": final_ME,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=20, help="untimed sweeps first")
    ap.add_argument("--L", type=int, default=16384)
    ap.add_argument("--beta", type=float, default=BETA_C)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--kernel-sweeps", type=int, default=50, help="sweeps timed launch by launch")
    ap.add_argument("--cpu-sweeps", type=int, default=8, help="sweeps in the CPU-oracle sample")
    ap.add_argument("--layout", choices=["fused", "int8", "packed"], default="fused",
                    help="fused: int8, both colours per launch, two buffers (default); int8: one launch "
                         "per colour, in place; packed: 1-bit spins, one launch per colour")
    ap.add_argument("--compare", type=int, default=1,
                    help="with the fused layout, also time the other two layouts on the same workload")
    ap.add_argument("--form", choices=["plain", "precision", "batch", "3d"], default="plain",
                    help="plain: the timed sweep (default); precision: bfloat16/half vs exact chains on "
                         "the --L lattice; batch: the 255-replica Binder-crossing run in one launch; "
                         "3d: the cubic lattice (--L3, default 1024) at the 3-D critical coupling")
    ap.add_argument("--L3", type=int, default=1024, help="edge of the cubic lattice for --form 3d")
    ap.add_argument("--meas", type=int, default=None, help="measurement sweeps of the precision/batch forms")
    ap.add_argument("--therm", type=int, default=None, help="thermalisation sweeps of the precision/batch forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run this many plain device copies of an L^2-byte buffer (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(one periodic lattice per GPU, no sharding).", file=sys.stderr)
        return 2

    import torch
    from paper_1903_11714_amd import ising

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    L, beta, seed, K, W = args.L, args.beta, args.seed, args.steps, args.warmup
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.form == "3d":
        print(json.dumps(bench_3d(ising, torch, args, stream)), flush=True)
        return 0
    if args.form != "plain":
        from paper_1903_11714_amd import studies
        if args.form == "precision":
            res = studies.precision_study(L=L, n_therm=args.therm if args.therm is not None else 1000,
                                          n_meas=args.meas if args.meas is not None else 10000, seed=seed)
        else:
            res = studies.batch_study(n_therm=args.therm if args.therm is not None else 2000,
                                      n_meas=args.meas if args.meas is not None else 20000)
        print(json.dumps({"form": args.form, **res}), flush=True)
        return 0

    if args.layout == "fused" and K % 2:
        K += 1  # whole two-sweep passes
        print(f"bench: fused layout times an even number of sweeps: {K}", file=sys.stderr, flush=True)
    if args.layout == "fused" and L > FUSED_MAX_L:
        print(f"bench: L={L} is above the fused sweep's limit ({FUSED_MAX_L}); timing the int8 layout",
              file=sys.stderr, flush=True)
        args.layout = "int8"
    main = run_layout(ising, torch, args.layout, L, beta, seed, K, W, args.kernel_sweeps, stream)
    lat_bytes = L * L // 8 if args.layout == "packed" else L * L
    alg_bytes = algorithmic_bytes(args.layout, L)
    achieved = alg_bytes / (main["avg_launch_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.layout, L)
    layout_text = {
        "fused": f"int8 layout, two sweeps per launch, lattice + scratch buffer ({2 * lat_bytes / 2**20:.0f} MiB)",
        "int8": f"int8 layout, one launch per colour, in place ({lat_bytes / 2**20:.0f} MiB)",
        "packed": f"1-bit layout, one launch per colour ({lat_bytes / 2**20:.0f} MiB)",
    }[args.layout]

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
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": KERNEL_NAME[args.layout],
            "avg_launch_us": main["avg_launch_ms"] * 1e3,
            "untraced_launch_us": main["untraced_launch_ms"] * 1e3,
            "alg_bytes_per_launch": alg_bytes,
            "sweeps_per_launch": FUSED_SWEEPS_PER_LAUNCH if args.layout == "fused" else 0.5,
        },
        "gpu_event_ms": main["gpu_ms"],
        "final_ME": main["final_ME"],
    }
    # The bound is the resource the kernel uses the larger share of: HBM (algorithmic bytes per
    # launch over the launch time) or the vector ALU (its VALU instructions per launch, from the
    # committed counters, over the launch time); the other one is reported beside it.
    alu = alu_roofline(args.layout, L, main["avg_launch_ms"])
    if alu is not None and alu["frac"] > result["roofline"]["frac"]:
        hbm = {k: result["roofline"].pop(k) for k in ("bound", "achieved", "peak", "unit", "frac")}
        rest = result["roofline"]
        result["roofline"] = {**{k: alu[k] for k in ("bound", "achieved", "peak", "unit", "frac")}, **rest,
                              "valu_busy": alu["valu_busy"], "valu_insts_per_launch": alu["valu_insts_per_launch"],
                              "hbm": hbm}
    elif alu is not None:
        result["roofline"]["alu"] = alu
    # context for the roofline: a plain device-to-device copy of an L^2-byte buffer (out of place,
    # as the fused sweep moves its bytes) on the same GPU
    cb = copy_bandwidth(torch, L, stream)
    result["roofline"]["copy_GBs"] = cb
    result["roofline"]["copy_kind"] = "out of place"
    result["roofline"]["hbm_frac_of_copy"] = achieved / cb if cb else None
    if args.compare and args.layout == "fused":
        # the same workload with the acceptance test in bfloat16 and in half (the chain differs:
        # u < p with both rounded to the format), on the same fused kernel
        for fmt in ("bf16", "fp16"):
            low = run_layout(ising, torch, "fused", L, beta, seed, K, W, args.kernel_sweeps, stream, fmt=fmt)
            gbs = alg_bytes / (low["avg_launch_ms"] * 1e-3) / 1e9
            result[f"{fmt}_accept"] = {
                "value": low["value"], "unit": "attempts/ns", "steps": K, "kernel": KERNEL_NAME["fused"],
                "avg_launch_us": low["avg_launch_ms"] * 1e3, "hbm_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                "vs_exact": low["value"] / main["value"], "final_ME": low["final_ME"],
            }
        # the same workload on the other layouts (same chain, bit-identical spins), for reference
        ks = max(K // 4, 1)
        for lay in ("int8", "packed"):
            other = run_layout(ising, torch, lay, L, beta, seed, ks, W, args.kernel_sweeps, stream)
            gbs = algorithmic_bytes(lay, L) / (other["avg_launch_ms"] * 1e-3) / 1e9
            result[f"{lay}_layout"] = {
                "value": other["value"], "unit": "attempts/ns", "steps": ks, "kernel": KERNEL_NAME[lay],
                "avg_launch_us": other["avg_launch_ms"] * 1e3,
                "hbm_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            }
    if args.copy_calibration:
        calibration_copies(torch, L * L, args.copy_calibration)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(L, beta, seed, args.cpu_sweeps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
