"""The two comparison studies of the forms beside the plain exact chain, run on the GPU.

precision_study (the paper's bfloat16 claim, Sec. 4.1): one long chain per (temperature,
acceptance format) on an L x L lattice; <|m|>, <e> and the Binder cumulant U4 with
autocorrelation-corrected errors; z-scores of bfloat16 and half against the exact chain, and of
every chain against Onsager's energy and Yang's magnetisation where those hold.

batch_study (the paper's U4(T) curves for several L, Sec. 4.1): every (L, T) replica in one
persistent launch; U4 per replica with jackknife errors and the temperature where the U4 curves
of neighbouring sizes cross, against T_c.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import analysis as A
from . import ising


def _chain_stats(trace: np.ndarray, n_sites: int) -> dict:
    m = trace[:, 0].astype(np.float64) / n_sites
    e = trace[:, 1].astype(np.float64) / n_sites
    am, am_err, am_tau = A.mean_err(np.abs(m))
    em, em_err, em_tau = A.mean_err(e)
    n_blocks = max(10, min(50, trace.shape[0] // max(1, int(4 * max(am_tau, em_tau)))))
    u4, u4_err = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=n_blocks)
    return {"abs_m": am, "abs_m_err": am_err, "tau_abs_m": am_tau, "e": em, "e_err": em_err, "tau_e": em_tau,
            "U4": u4, "U4_err": u4_err}


def precision_study(L: int = 16384, temps=(2.0, A.T_C, 2.5), n_therm: int = 1000, n_meas: int = 10000,
                    formats=("exact", "bf16", "fp16"), seed: int = 1, device: str = "cuda") -> dict:
    """Runs len(temps) x len(formats) chains on the packed layout (identical to int8)."""
    import torch
    out = {"L": L, "n_therm": n_therm, "n_meas": n_meas, "seed": seed, "runs": []}
    t_start = time.perf_counter()
    for T in temps:
        beta = 1.0 / T
        cold = T < A.T_C          # ordered phase: start from the ordered state (a hot start only coarsens)
        row = {"T": T, "beta": beta, "start": "cold" if cold else "hot", "formats": {}}
        for fmt in formats:
            planes = ising.new_packed(L, None if cold else seed, device=device)
            ising.ising_sweep_packed_fmt(planes, L, beta, fmt, n_therm, seed, 0)
            trace = torch.empty((n_meas, 2), dtype=torch.int64, device=device)
            ising.ising_sweep_packed_fmt(planes, L, beta, fmt, n_meas, seed, n_therm, trace)
            mom = torch.empty(5, dtype=torch.float64, device=device)
            ising.ising_moments(trace, n_meas, L * L, mom)
            tr = trace.cpu().numpy()
            st = _chain_stats(tr, L * L)
            st["fp64_moments"] = dict(zip(["abs_m", "m2", "m4", "e", "e2"], mom.cpu().tolist()))
            st["U4_from_fp64_moments"] = A.binder(st["fp64_moments"]["m2"], st["fp64_moments"]["m4"])
            row["formats"][fmt] = st
            del planes, trace
        ex = row["formats"].get("exact")
        for fmt, st in row["formats"].items():
            zs = {}
            if ex is not None and fmt != "exact":
                zs["vs_exact"] = {k: A.z(st[k], st[k + "_err"], ex[k], ex[k + "_err"]) for k in ("abs_m", "e", "U4")}
            if abs(T - A.T_C) > 0.05:
                zs["e_vs_onsager"] = A.z(st["e"], st["e_err"], A.onsager_energy(beta), 0.0)
                if T < A.T_C:
                    zs["abs_m_vs_yang"] = A.z(st["abs_m"], st["abs_m_err"], A.yang_magnetisation(beta), 0.0)
            st["z"] = zs
        out["runs"].append(row)
    out["seconds"] = time.perf_counter() - t_start
    return out


def find_crossings(Ls, temps, u4) -> list:
    """Temperature where the U4 curves of neighbouring sizes a < b cross.  Above T_c the smaller
    lattice has the larger U4, below it the smaller one, so the crossing is a sign change of
    U4_a - U4_b from <= 0 to > 0 with rising T.  On the plateaus (U4 near 2/3 at low T, near 0 at
    high T) the difference is noise and changes sign by chance; the crossing taken is the sign change
    whose two bracketing differences are largest in units of their errors.  Linear interpolation;
    error from the bracketing points' errors over the slope."""
    temps = np.asarray(temps, dtype=np.float64)
    out = []
    for a, b in zip(Ls[:-1], Ls[1:]):
        va, ea = (np.asarray(x, dtype=np.float64) for x in u4[a])
        vb, eb = (np.asarray(x, dtype=np.float64) for x in u4[b])
        d, de = va - vb, np.sqrt(ea ** 2 + eb ** 2)
        best = None
        for k in range(len(temps) - 1):
            if d[k] <= 0 < d[k + 1]:
                sig = (abs(d[k]) + abs(d[k + 1])) / max(de[k] + de[k + 1], 1e-300)
                if best is None or sig > best[0]:
                    best = (sig, k)
        if best is None:
            out.append({"pair": [a, b], "T_cross": None})
            continue
        sig, k = best
        slope = (d[k + 1] - d[k]) / (temps[k + 1] - temps[k])
        t_star = temps[k] - d[k] / slope
        err = float(max(de[k], de[k + 1]) / abs(slope))
        out.append({"pair": [a, b], "T_cross": float(t_star), "err": err, "significance": float(sig),
                    "z_vs_Tc": float((t_star - A.T_C) / err) if err > 0 else None})
    return out


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
    # first call tunes the workgroup size on this table (a short run the real one overwrites)
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
    u4 = {}
    for L in Ls:
        vals, errs = [], []
        for _ in temps:
            m = tr[idx, :, 0].astype(np.float64) / (L * L)
            est, err = A.jackknife(A.binder, [m * m, m ** 4], n_blocks=50)
            vals.append(est)
            errs.append(err)
            idx += 1
        u4[L] = (np.array(vals), np.array(errs))
        res["curves"][str(L)] = {"U4": vals, "U4_err": errs,
                                 "abs_m": [float(x) for x in mo[idx - len(temps):idx, 0]]}
    res["crossings"] = find_crossings(Ls, temps, u4)
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
