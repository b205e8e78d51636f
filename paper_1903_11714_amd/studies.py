"""The two comparison studies of the forms beside the plain exact chain, run on the GPU.

precision_study (the paper's bfloat16 claim, Sec. 4.1, Fig. 3): for each temperature, several
seeds, and for each seed one chain per acceptance format (exact, bfloat16, half) on an L x L
lattice.  The low-precision chains use the SAME random numbers as the exact chain of their seed, so
the two are correlated; the comparison therefore works on paired differences:

* per seed, the difference of the time averages of |m| and e with the error of the difference
  series itself (its own tau_int), and the difference of U4 with a jackknife over the same time
  blocks of both chains;
* over seeds, the mean of the per-seed differences with its standard error across the independent
  seeds (ddof = 1).  This one holds whether or not a chain is in equilibrium (at T_c a single chain
  of L = 16384 is not: tau grows like L^2.17), since every seed runs the same protocol.

Each chain's own averages (seed means with their across-seed errors) are compared with Onsager's
energy and Yang's magnetisation where those hold (T away from T_c).

batch_study (the paper's U4(T) curves for several L, Sec. 4.1): every (L, T) replica in one
persistent launch; U4 per replica with jackknife errors, per-replica integrated autocorrelation
times (flagged where a replica ran fewer than 50 tau), and the temperature where the U4 curves of
neighbouring sizes cross, with a jackknife error over synchronised blocks of every replica.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import analysis as A
from . import ising

OBS = ("abs_m", "e", "U4")


def _series(trace: np.ndarray, n_sites: int):
    m = trace[:, 0].astype(np.float64) / n_sites
    e = trace[:, 1].astype(np.float64) / n_sites
    return m, e


def _n_blocks(n: int, tau: float) -> int:
    """Jackknife blocks: each block spans at least 4 tau_int where the series allows, 10 .. 50 blocks."""
    return max(10, min(50, n // max(1, int(4 * tau))))


def chain_stats(trace: np.ndarray, n_sites: int) -> dict:
    m, e = _series(trace, n_sites)
    am, am_err, am_tau = A.mean_err(np.abs(m))
    em, em_err, em_tau = A.mean_err(e)
    u4, u4_err = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=_n_blocks(m.size, max(am_tau, em_tau)))
    return {"abs_m": am, "abs_m_err": am_err, "tau_abs_m": am_tau, "e": em, "e_err": em_err, "tau_e": em_tau,
            "U4": u4, "U4_err": u4_err}


def paired_stats(trace: np.ndarray, ref: np.ndarray, n_sites: int) -> dict:
    """Differences (this chain - reference chain) of the time averages, with errors from the paired
    difference series (the two chains share their random numbers)."""
    m, e = _series(trace, n_sites)
    m0, e0 = _series(ref, n_sites)
    d_am, d_am_err, tau_am = A.paired_mean_err(np.abs(m), np.abs(m0))
    d_e, d_e_err, tau_e = A.paired_mean_err(e, e0)
    nb = _n_blocks(m.size, max(tau_am, tau_e))
    d_u4, d_u4_err = A.paired_jackknife(A.binder, [m * m, m ** 4], [m0 * m0, m0 ** 4], n_blocks=nb)
    return {"abs_m": d_am, "abs_m_err": d_am_err, "tau_abs_m": tau_am, "e": d_e, "e_err": d_e_err, "tau_e": tau_e,
            "U4": d_u4, "U4_err": d_u4_err}


def _z(d: float, err: float):
    return d / err if err and err > 0 and math.isfinite(err) else None


def precision_study(L: int = 16384, temps=(2.0, A.T_C, 2.5), n_therm: int = 1000, n_meas: int = 10000,
                    formats=("exact", "bf16", "fp16"), seeds=tuple(range(1, 9)), device: str = "cuda",
                    log=None) -> dict:
    """len(temps) x len(seeds) x len(formats) chains on the packed layout (bit-identical to int8).
    Below T_c every chain starts ordered (a hot start there only coarsens), elsewhere hot."""
    import torch
    assert formats[0] == "exact"
    N = L * L
    out = {"L": L, "n_therm": n_therm, "n_meas": n_meas, "seeds": list(seeds), "formats": list(formats),
           "layout": "packed (1-bit), identical chain to int8", "runs": []}
    t_start = time.perf_counter()
    for T in temps:
        beta = 1.0 / T
        cold = T < A.T_C
        traces = {fmt: [] for fmt in formats}
        for seed in seeds:
            for fmt in formats:
                planes = ising.new_packed(L, None if cold else seed, device=device)
                ising.ising_sweep_packed_fmt(planes, L, beta, fmt, n_therm, seed, 0)
                trace = torch.empty((n_meas, 2), dtype=torch.int64, device=device)
                ising.ising_sweep_packed_fmt(planes, L, beta, fmt, n_meas, seed, n_therm, trace)
                traces[fmt].append(trace.cpu().numpy())
                del planes, trace
            if log:
                log(f"precision: T={T:.4f} seed {seed} done")
        row = {"T": T, "beta": beta, "start": "cold" if cold else "hot", "formats": {}}
        for fmt in formats:
            per_seed = [chain_stats(tr, N) for tr in traces[fmt]]
            agg = {}
            for k in OBS:
                mean, err = A.seed_mean_err([s[k] for s in per_seed])
                agg[k] = mean
                agg[k + "_err_seeds"] = err
            agg["tau_abs_m"] = [s["tau_abs_m"] for s in per_seed]
            agg["tau_e"] = [s["tau_e"] for s in per_seed]
            if abs(T - A.T_C) > 0.05:
                agg["z_e_vs_onsager"] = _z(agg["e"] - A.onsager_energy(beta), agg["e_err_seeds"])
                if T < A.T_C:
                    agg["z_abs_m_vs_yang"] = _z(agg["abs_m"] - A.yang_magnetisation(beta), agg["abs_m_err_seeds"])
            if fmt != "exact":
                pairs = [paired_stats(tr, ref, N) for tr, ref in zip(traces[fmt], traces["exact"])]
                vs = {}
                for k in OBS:
                    diffs = [p[k] for p in pairs]
                    d, d_err = A.seed_mean_err(diffs)
                    # tau-corrected errors of the per-seed paired differences, combined over seeds
                    pooled = math.sqrt(sum(p[k + "_err"] ** 2 for p in pairs)) / len(pairs)
                    vs[k] = {"diff": d, "err_seeds": d_err, "z_seeds": _z(d, d_err),
                             "err_paired_tau": pooled, "z_paired_tau": _z(d, pooled),
                             "per_seed": [{"diff": p[k], "err": p[k + "_err"]} for p in pairs]}
                agg["vs_exact"] = vs
            agg["per_seed"] = per_seed
            row["formats"][fmt] = agg
        out["runs"].append(row)
    out["seconds"] = time.perf_counter() - t_start
    return out


def precision_table(rec: dict) -> str:
    """Markdown z-table of a precision_study record."""
    lines = [f"L = {rec['L']}, {rec['n_therm']} + {rec['n_meas']} sweeps per chain, seeds {rec['seeds'][0]}.."
             f"{rec['seeds'][-1]} ({len(rec['seeds'])} per format), {rec['layout']}.", "",
             "| T | start | format | <\\|m\\|> | <e> | U4 | z vs exact over seeds (\\|m\\|, e, U4) | "
             "z vs exact, paired tau-corrected (\\|m\\|, e, U4) | z: e vs Onsager | z: \\|m\\| vs Yang |",
             "|---|---|---|---|---|---|---|---|---|---|"]

    def f(v, nd=3):
        return "—" if v is None else f"{v:.{nd}f}" if abs(v) < 1e4 else f"{v:.3g}"

    for row in rec["runs"]:
        for fmt, a in row["formats"].items():
            vs = a.get("vs_exact")
            zs = ", ".join(f(vs[k]["z_seeds"], 1) for k in OBS) if vs else "—"
            zp = ", ".join(f(vs[k]["z_paired_tau"], 1) for k in OBS) if vs else "—"
            lines.append(
                f"| {row['T']:.4f} | {row['start']} | {fmt} | {a['abs_m']:.6f} ± {a['abs_m_err_seeds']:.6f} | "
                f"{a['e']:.7f} ± {a['e_err_seeds']:.7f} | {a['U4']:.4f} ± {a['U4_err_seeds']:.4f} | {zs} | {zp} | "
                f"{f(a.get('z_e_vs_onsager'), 1)} | {f(a.get('z_abs_m_vs_yang'), 1)} |")
    return "\n".join(lines)


def config5_replicas(Ls=(32, 64, 128, 256, 512), n_temps: int = 51, t_lo: float = 2.0, t_hi: float = 2.6,
                     seed0: int = 1000):
    temps = np.linspace(t_lo, t_hi, n_temps)
    reps = []
    for L in Ls:
        for T in temps:
            reps.append((L, 1.0 / float(T), seed0 + len(reps)))
    return reps, temps


def _schedule(reps) -> tuple[int, int, int, int]:
    """The batch schedule in use: the tuned one, or the one the options fix."""
    try:
        return ising.ising_batch_schedule(reps)
    except ising.IsingError:
        return tuple(ising.ising_get_option(k)
                     for k in ("batch_threads", "batch_slab_sites", "batch_depth", "batch_lists_per_cu"))


def batch_study(Ls=(32, 64, 128, 256, 512), n_temps: int = 51, n_therm: int = 2000, n_meas: int = 20000,
                fmt="exact", device: str = "cuda", check_plain: int = 4, start: int = 3) -> dict:
    """start 3: replicas below T_c begin ordered (all +1), the others from their hot start."""
    import torch
    reps, temps = config5_replicas(Ls, n_temps)
    ws = torch.empty(ising.ising_batch_workspace_bytes(reps), dtype=torch.uint8, device=device)
    # first call tunes the schedule on this table (a short run the real one overwrites)
    ising.batch_run(reps, 2, 1, fmt=fmt, workspace=ws, start=start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    moments, trace, ws = ising.batch_run(reps, n_therm, n_meas, fmt=fmt, workspace=ws, start=start)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    attempts = float(sum(L * L for L, _, _ in reps)) * (n_therm + n_meas)
    tr = trace.cpu().numpy()
    mo = moments.cpu().numpy()
    res = {"Ls": list(Ls), "temps": [float(t) for t in temps], "n_therm": n_therm, "n_meas": n_meas,
           "replicas": len(reps), "seconds": wall, "attempts_per_ns": attempts / (wall * 1e9),
           "schedule": dict(zip(("threads", "slab_sites", "depth", "lists_per_cu"), _schedule(reps))), "curves": {}}
    idx = 0
    m_series = {}
    tau_limit = n_meas / 50.0
    flagged = []
    for L in Ls:
        vals, errs, taus = [], [], []
        m_series[L] = []
        for T in temps:
            m = tr[idx, :, 0].astype(np.float64) / (L * L)
            m_series[L].append(m)
            tau = max(A.tau_int(np.abs(m)), A.tau_int(m * m))
            est, err = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=50)
            vals.append(est)
            errs.append(err)
            taus.append(tau)
            if tau > tau_limit:
                flagged.append({"L": L, "T": float(T), "tau_int": tau})
            idx += 1
        res["curves"][str(L)] = {"U4": vals, "U4_err": errs, "tau_int_m": taus,
                                 "abs_m": [float(x) for x in mo[idx - len(temps):idx, 0]]}
    res["tau_limit"] = tau_limit
    res["tau_flagged"] = flagged
    # jackknife blocks of at least four tau_int of the slowest replica at each crossing
    res["crossings"] = A.u4_crossings(Ls, temps, m_series, n_blocks=A.crossing_blocks)
    # the batched replicas are the plain chain: re-run one replica of every size >= 64 (the
    # middle of its temperature range) with the single-lattice path and compare the traces
    checks = []
    for j, L in enumerate(Ls):
        if L < 64 or len(checks) >= check_plain:
            continue
        k = j * len(temps) + len(temps) // 2
        _, beta, seed = reps[k]
        p = ising.new_packed(L, seed, device=device)
        t = torch.empty((n_meas, 2), dtype=torch.int64, device=device)
        ising.ising_sweep_packed_fmt(p, L, beta, fmt, n_therm, seed, 0)
        ising.ising_sweep_packed_fmt(p, L, beta, fmt, n_meas, seed, n_therm, t)
        checks.append({"replica": k, "L": L, "T": 1.0 / beta, "identical_trace": bool(torch.equal(t, trace[k]))})
    res["plain_path_checks"] = checks
    return res


def batch_table(rec: dict) -> str:
    """Markdown summary of a batch_study record: throughput, crossings, tau diagnostics."""
    lines = [f"{rec['replicas']} replicas, L in {rec['Ls']}, {len(rec['temps'])} temperatures on "
             f"[{rec['temps'][0]:.3f}, {rec['temps'][-1]:.3f}], {rec['n_therm']} + {rec['n_meas']} sweeps: "
             f"{rec['seconds']:.3f} s, {rec['attempts_per_ns']:.0f} attempts/ns; schedule {rec['schedule']}.", "",
             "| pair | T_cross ± jackknife | z vs T_c | quadratic interpolation | ± interpolation | z (both errors) "
             "| bracket | jackknife blocks |", "|---|---|---|---|---|---|---|---|"]
    for c in rec["crossings"]:
        if c.get("T_cross") is None:
            lines.append(f"| {c['pair']} | none | — | — | — | — | — | — |")
        else:
            z, zt = c.get("z_vs_Tc"), c.get("z_total")
            quad = c.get("T_cross_quad")
            lines.append(f"| {c['pair'][0]}, {c['pair'][1]} | {c['T_cross']:.4f} ± {c['err']:.4f} | "
                         f"{'—' if z is None else f'{z:.1f}'} | {'—' if quad is None else f'{quad:.4f}'} | "
                         f"{'—' if quad is None else format(c['syst'], '.4f')} | {'—' if zt is None else f'{zt:.1f}'} | "
                         f"{c['bracket'][0]:.3f}–{c['bracket'][1]:.3f} | {c['n_blocks']} |")
    lines += ["", f"Replicas with tau_int(|m| or m^2) above n_meas / 50 = {rec['tau_limit']:.0f} sweeps: "
              f"{len(rec['tau_flagged'])} of {rec['replicas']}"]
    by_L = {}
    for f in rec["tau_flagged"]:
        by_L.setdefault(f["L"], []).append(f)
    for L, fl in sorted(by_L.items()):
        lines.append(f"- L = {L}: {len(fl)} replicas, T {min(x['T'] for x in fl):.3f}–{max(x['T'] for x in fl):.3f}, "
                     f"tau_int up to {max(x['tau_int'] for x in fl):.0f}")
    return "\n".join(lines)
