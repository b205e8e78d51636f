"""Writes config2_window_L16384_n1000.json: the oracle's view of the benchmark's own run.

The run: a periodic 16384 x 16384 lattice, hot start from seed 1, beta_c = ln(1 + sqrt 2) / 2,
1000 sweeps from sweep index 0 (white then black half-sweeps, Sec. 3.1).  After n sweeps a site
depends only on the sites within distance 2n (one site per colour update), so the oracle runs a
(2048 + 4n)^2 window of the torus with global Philox counters and keeps the central 2048 x 2048
block (oracle.crop).  The block is taken across both seams of the torus (rows and columns
L - 1024 .. L + 1023, wrapped).  The fixture stores its SHA-256 (int8 bytes, row-major) and a few
sums, so the GPU test can compare the whole block without storing it.

Calls only oracle/ (about five minutes on 8 host threads): python tests/golden/make_config2_window.py
"""
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402

L, SEED, N, OFFSET = 16384, 1, 1000, 0
BETA = 0.5 * math.log1p(math.sqrt(2.0))
R0 = C0 = L - 1024
H = W = 2048


def main() -> None:
    t0 = time.perf_counter()
    block = oracle.crop(L, SEED, BETA, N, OFFSET, R0, C0, H, W)
    dt = time.perf_counter() - t0
    assert block.dtype == np.int8 and block.shape == (H, W)
    assert np.all((block == 1) | (block == -1))
    rec = {
        "what": "oracle.crop of the 16384^2 benchmark run after 1000 sweeps, 2048^2 block across both seams",
        "L": L, "seed": SEED, "beta": BETA, "n_sweeps": N, "sweep_offset": OFFSET,
        "r0": R0, "c0": C0, "h": H, "w": W,
        "sha256_int8_row_major": hashlib.sha256(np.ascontiguousarray(block).tobytes()).hexdigest(),
        "sum": int(block.astype(np.int64).sum()),
        "first_row_sum": int(block[0].astype(np.int64).sum()),
        "first_col_sum": int(block[:, 0].astype(np.int64).sum()),
        "bond_sum": int((block[:, :-1].astype(np.int64) * block[:, 1:]).sum() +
                        (block[:-1, :].astype(np.int64) * block[1:, :]).sum()),
        "generator": "tests/golden/make_config2_window.py (calls oracle.crop only)",
        "oracle_seconds": round(dt, 1),
        "oracle_threads": oracle.num_threads(),
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_window_L16384_n1000.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
