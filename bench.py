#!/usr/bin/env python3
"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

Workload (the paper's single-lattice measurement, Sec. 4.2: time per sweep of all black and
all white sites, flips/ns = L^2 / sweep time): a periodic 16384 x 16384 int8 lattice, hot
start from seed 1, beta = beta_c = ln(1 + sqrt 2) / 2, exact-threshold acceptance, with the
(M, E) trace recorded after every sweep.  One "step" is one sweep.  The lattice is resident in
HBM before the timed region starts.

Prints one JSON line with the throughput (spin-flip attempts per ns), the roofline of the
dominant kernel (the half-sweep kernel; algorithmic bytes = one read and one write of the
L^2-byte lattice per launch, measured with HIP events on the launch stream) and the CPU
oracle's throughput on a bounded sample of the same workload.
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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1903_11714_amd", "csrc", f) for f in ("ising.hip", "philox.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(layout: str, L: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get(f"{layout}_L{L}")
    if not entry or entry.get("source_hash") != kernel_source_hash():
        return None
    return entry.get("hbm_bytes_per_launch")


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


def run_layout(ising, torch, layout, L, beta, seed, K, W, kernel_sweeps, stream):
    """Hot start, W warm-up sweeps, K timed sweeps with the (M, E) trace, then `kernel_sweeps`
    sweeps with every half-sweep launch bracketed by events."""
    dev = torch.device("cuda:0")
    if layout == "int8":
        lat = torch.empty((L, L), dtype=torch.int8, device=dev)
        ising.ising_init(lat, L, seed, stream)
        sweep, half = ising.ising_sweep, ising.ising_half_sweep
    else:
        lat = torch.empty(L * L // 32, dtype=torch.int32, device=dev)
        ising.ising_init_packed(lat, L, seed, stream)
        sweep, half = ising.ising_sweep_packed, ising.ising_half_sweep_packed
    warm_trace = torch.empty((max(W, 1), 2), dtype=torch.int64, device=dev)
    trace = torch.empty((max(K, 1), 2), dtype=torch.int64, device=dev)
    if W:
        sweep(lat, L, beta, W, seed, 0, warm_trace, stream)
    torch.cuda.synchronize()
    print(f"bench: {layout} L={L} warmup={W} done", file=sys.stderr, flush=True)

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sweep(lat, L, beta, K, seed, W, trace, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    print(f"bench: {layout} timed {K} sweeps in {wall:.3f} s wall, {gpu_ms:.1f} ms events", file=sys.stderr,
          flush=True)
    final_ME = trace[K - 1].tolist() if K else None

    # dominant kernel: each half-sweep launch bracketed by events on the launch stream
    nk = kernel_sweeps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nk + 1)]
    t = W + K
    evs[0].record(stream)
    for i in range(nk):
        half(lat, L, beta, seed, t + i, 1, stream)
        evs[2 * i + 1].record(stream)
        half(lat, L, beta, seed, t + i, 0, stream)
        evs[2 * i + 2].record(stream)
    torch.cuda.synchronize()
    durs = [evs[k].elapsed_time(evs[k + 1]) for k in range(2 * nk)]
    del lat
    return {
        "value": float(L) * L * K / (wall * 1e9),
        "wall_s": wall,
        "gpu_ms": gpu_ms,
        "avg_launch_ms": sum(durs) / len(durs),
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
    ap.add_argument("--layout", choices=["int8", "packed"], default="int8")
    ap.add_argument("--compare-packed", type=int, default=1,
                    help="with the int8 layout, also time the 1-bit layout on the same workload")
    ap.add_argument("--form", choices=["plain", "precision", "batch"], default="plain",
                    help="plain: the timed sweep (default); precision: bfloat16/half vs exact chains on "
                         "the --L lattice; batch: the 255-replica Binder-crossing run in one launch")
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

    main = run_layout(ising, torch, args.layout, L, beta, seed, K, W, args.kernel_sweeps, stream)
    lat_bytes = L * L if args.layout == "int8" else L * L // 8
    # int8: each launch reads and writes the L^2-byte lattice.  packed: each launch reads both
    # colour planes (L^2 / 8 bytes) and writes one (L^2 / 16 bytes).
    alg_bytes = 2.0 * L * L if args.layout == "int8" else 3.0 * L * L / 16.0
    achieved = alg_bytes / (main["avg_launch_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.layout, L)

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
        "dtype": "int8" if args.layout == "int8" else "u32 (1-bit spins)",
        "data": "synthetic: Philox hot start from the seed (no dataset)",
        "config": {
            "workload": f"single periodic {L}x{L} lattice, beta={beta:.6g}"
                        f"{' (T_c)' if abs(beta - BETA_C) < 1e-12 else ''}, hot start seed {seed}, plain "
                        f"exact-threshold checkerboard Metropolis, {args.layout} layout "
                        f"({lat_bytes / 2**20:.0f} MiB), (M,E) traced every sweep",
            "L": L, "beta": beta, "layout": args.layout, "sweeps_timed": K,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_sweep_int8 (one colour per launch)" if args.layout == "int8"
                      else "k_sweep_packed (one colour per launch)",
            "avg_launch_us": main["avg_launch_ms"] * 1e3,
            "alg_bytes_per_launch": alg_bytes,
        },
        "gpu_event_ms": main["gpu_ms"],
        "final_ME": main["final_ME"],
    }
    if args.compare_packed and args.layout == "int8":
        # the same workload on the 1-bit layout (same chain, bit-identical spins), for reference
        ks = max(K // 4, 1)
        other = run_layout(ising, torch, "packed", L, beta, seed, ks, W, args.kernel_sweeps, stream)
        result["packed_layout"] = {
            "value": other["value"], "unit": "attempts/ns", "steps": ks,
            "avg_launch_us": other["avg_launch_ms"] * 1e3,
            "hbm_GBs": 3.0 * L * L / 16.0 / (other["avg_launch_ms"] * 1e-3) / 1e9,
        }
    if args.copy_calibration:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the
        # per-launch HBM traffic read from the same counters for the sweep kernel.
        # (int8 -> uint8 goes through an elementwise copy kernel that reads L^2 bytes and writes
        # L^2 bytes, like the sweep; a same-dtype copy would use the runtime's blit kernel.)
        src = torch.empty((L, L), dtype=torch.int8, device=dev)
        ising.ising_fill(src, L, 1, stream)
        dst = torch.empty((L, L), dtype=torch.uint8, device=dev)
        for _ in range(args.copy_calibration):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(L, beta, seed, args.cpu_sweeps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
