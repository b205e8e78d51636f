"""The error model of the precision study, checked on the oracle's own chains (CPU).

A bfloat16 chain and the exact chain of the same seed share every random number, so they are
positively correlated and their difference must take its error from the paired difference series.
Over independent seeds, the scatter of the per-seed differences is the truth the error must match.
"""
import math

import numpy as np
import pytest

from paper_1903_11714_amd import analysis as A
from paper_1903_11714_amd import studies as S


def _chain(oracle_lib, L, beta, fmt, seed, n_therm, n_meas):
    s = oracle_lib.init(L, seed)
    if fmt == "exact":
        oracle_lib.sweep(s, beta, n_therm, seed, 0)
        return oracle_lib.sweep(s, beta, n_meas, seed, n_therm, trace=True)
    oracle_lib.sweep_fmt(s, beta, fmt, n_therm, seed, 0)
    return oracle_lib.sweep_fmt(s, beta, fmt, n_meas, seed, n_therm, trace=True)


def test_paired_errors_match_the_scatter_over_seeds(oracle_lib):
    L, beta, n_therm, n_meas = 16, 0.4, 200, 4000
    N = L * L
    diffs, errs, quads = [], [], []
    for seed in range(1, 25):
        ex = _chain(oracle_lib, L, beta, "exact", seed, n_therm, n_meas)
        lo = _chain(oracle_lib, L, beta, "bf16", seed, n_therm, n_meas)
        p = S.paired_stats(lo, ex, N)
        a, b = S.chain_stats(lo, N), S.chain_stats(ex, N)
        diffs.append(p["e"])
        errs.append(p["e_err"])
        quads.append(math.hypot(a["e_err"], b["e_err"]))
    scatter = np.std(diffs, ddof=1)
    rms = math.sqrt(np.mean(np.square(errs)))
    # 24 seeds: the scatter itself is known to ~15%
    assert rms == pytest.approx(scatter, rel=0.3), (rms, scatter)
    # the shared random numbers correlate the chains: quadrature would overstate the error
    assert np.mean(quads) > 1.2 * rms


def test_precision_table_renders_a_record():
    per = {"abs_m": 0.5, "abs_m_err_seeds": 0.01, "e": -1.1, "e_err_seeds": 0.001, "U4": 0.3, "U4_err_seeds": 0.02}
    vs = {k: {"z_seeds": 1.5, "z_paired_tau": 2.5} for k in S.OBS}
    rec = {"L": 64, "n_therm": 10, "n_meas": 100, "seeds": [1, 2], "layout": "packed",
           "runs": [{"T": 2.5, "start": "hot", "formats": {"exact": dict(per), "bf16": dict(per, vs_exact=vs)}}]}
    text = S.precision_table(rec)
    assert text.count("\n| 2.5000 |") == 2 and "1.5, 1.5, 1.5" in text and "2.5, 2.5, 2.5" in text
