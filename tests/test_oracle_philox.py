"""Pin the oracle's Philox4x32-10 against rocRAND's independent open-source engine.

The paper draws one uniform per site per colour update (Sec. 3.2, Algorithm 1, "probs";
Sec. 5.1, random_uniform).  Both the oracle and the HIP path take those numbers from
Philox4x32-10 (Salmon et al., SC'11).  rocRAND ships a host-callable implementation of the
same function as header source; a tiny helper program evaluates it here.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("g++ or the rocRAND headers are not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-o", exe, HELPER], check=True)

    def run(rows: np.ndarray) -> np.ndarray:
        text = "\n".join(" ".join(str(int(v)) for v in row) for row in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)

    return run


def test_philox_matches_rocrand(oracle_lib, rocrand_ref):
    rng = np.random.default_rng(12345)
    rows = rng.integers(0, 2**32, size=(3000, 6), dtype=np.uint64)
    special = np.array([[0, 0, 0, 0, 0, 0],
                        [2**32 - 1] * 6,
                        [1, 0, 0, 0, 0, 0],
                        [0, 0, 0, 1, 0, 0],
                        [0, 0, 0, 0, 0, 1],
                        [7, 16383, 999, 15, 1, 0]], dtype=np.uint64)
    rows = np.concatenate([special, rows])
    ref = rocrand_ref(rows)
    got = np.array([oracle_lib.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_philox_is_a_bijection_on_small_sample(oracle_lib):
    # Different counters under one key never collide (Philox is a bijection of the counter).
    outs = {tuple(oracle_lib.philox4x32_10([i, 0, 0, 0], [1, 0])) for i in range(5000)}
    assert len(outs) == 5000
