"""CPU oracle for the checkerboard Metropolis sweep of the periodic 2D Ising model.

TEST INFRASTRUCTURE ONLY.  The plain C implementation lives in ``ising_oracle.c``; this
module builds it with gcc and exposes it through ctypes.  Only the tests, the smoke entry
point and the benchmark's CPU-baseline leg may import it; the product path never does.

Paper: arXiv 1903.11714 (Yang et al.).  Sec. 3 (Hamiltonian, torus), Sec. 3.1 (checkerboard
decomposition and the white-then-black order), Sec. 3.2 Algorithm 1 (neighbour sum, uniform
below the acceptance ratio, flip), Sec. 4.1 (magnetisation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ising_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True, out: str | None = None, native: bool = False) -> str:
    """Compile the oracle.  Default: ``oracle/liboracle.so`` with -O2 and no -march, so the library
    built once runs on whichever host runs the tests.  native=True: -O3 -march=native into ``out``
    (a copy for timing on the host that builds it; same source, same results)."""
    lib = out or _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp%d" % os.getpid()
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        cmd = ["gcc", *opt, "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


def load_native(directory: str) -> str:
    """Build the -O3 -march=native copy into `directory` and use it for every later call (the CPU
    baseline's timing).  Returns the compiler flags used."""
    global _lib
    path = build(force=True, out=os.path.join(directory, "liboracle_native.so"), native=True)
    _lib = _configure(ctypes.CDLL(path))
    return "gcc -O3 -march=native -fopenmp"


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(lib):
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i8p = ctypes.POINTER(ctypes.c_int8)
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_int]
    lib.oracle_uniform.restype = ctypes.c_uint32
    lib.oracle_thresholds.argtypes = [ctypes.c_double, u64p]
    lib.oracle_thresholds.restype = None
    lib.oracle_init_site.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_init_site.restype = ctypes.c_int
    lib.oracle_init.argtypes = [i8p, ctypes.c_int64, ctypes.c_uint64]
    lib.oracle_init.restype = None
    lib.oracle_local_field.argtypes = [i8p, ctypes.c_int64, i8p]
    lib.oracle_local_field.restype = None
    lib.oracle_half_sweep.argtypes = [i8p, ctypes.c_int64, u64p, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_int]
    lib.oracle_half_sweep.restype = None
    lib.oracle_sweep.argtypes = [i8p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                                 ctypes.c_uint64, ctypes.c_uint64, i64p]
    lib.oracle_sweep.restype = None
    lib.oracle_observables.argtypes = [i8p, ctypes.c_int64, i64p]
    lib.oracle_observables.restype = None
    lib.oracle_crop.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_int64, i8p]
    lib.oracle_crop.restype = None
    lib.oracle_round_fmt.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.oracle_round_fmt.restype = ctypes.c_double
    lib.oracle_p_fmt.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.oracle_p_fmt.restype = ctypes.c_double
    lib.oracle_u_fmt.argtypes = [ctypes.c_uint32, ctypes.c_int]
    lib.oracle_u_fmt.restype = ctypes.c_double
    lib.oracle_sweep_fmt.argtypes = [i8p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                     ctypes.c_uint64, ctypes.c_uint64, i64p]
    lib.oracle_sweep_fmt.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_moments.argtypes = [i64p, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_moments.restype = None
    lib.oracle3_thresholds.argtypes = [ctypes.c_double, u64p]
    lib.oracle3_thresholds.restype = None
    lib.oracle3_init.argtypes = [i8p, ctypes.c_int64, ctypes.c_uint64]
    lib.oracle3_init.restype = None
    lib.oracle3_local_field.argtypes = [i8p, ctypes.c_int64, i8p]
    lib.oracle3_local_field.restype = None
    lib.oracle3_half_sweep.argtypes = [i8p, ctypes.c_int64, u64p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
    lib.oracle3_half_sweep.restype = None
    lib.oracle3_sweep.argtypes = [i8p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_uint64, i64p]
    lib.oracle3_sweep.restype = None
    lib.oracle3_observables.argtypes = [i8p, ctypes.c_int64, i64p]
    lib.oracle3_observables.restype = None
    lib.oracle3_crop.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, i8p]
    lib.oracle3_crop.restype = None
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _lattice(spins: np.ndarray) -> np.ndarray:
    if spins.dtype != np.int8 or spins.ndim != 2 or spins.shape[0] != spins.shape[1]:
        raise ValueError("lattice must be a square int8 array")
    if not spins.flags.c_contiguous:
        raise ValueError("lattice must be C-contiguous")
    return spins


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                                 _ptr(out, ctypes.c_uint32))
    return out


def uniform(seed: int, r: int, c: int, t: int, q: int) -> int:
    return int(_load().oracle_uniform(seed, r, c, t, q))


def thresholds(beta: float) -> tuple[int, int]:
    T = np.zeros(2, dtype=np.uint64)
    _load().oracle_thresholds(float(beta), _ptr(T, ctypes.c_uint64))
    return int(T[0]), int(T[1])


def init_site(seed: int, r: int, c: int) -> int:
    return int(_load().oracle_init_site(seed, r, c))


def init(L: int, seed: int) -> np.ndarray:
    s = np.empty((L, L), dtype=np.int8)
    _load().oracle_init(_ptr(s, ctypes.c_int8), L, seed)
    return s


def local_field(spins: np.ndarray) -> np.ndarray:
    s = _lattice(spins)
    nn = np.empty_like(s)
    _load().oracle_local_field(_ptr(s, ctypes.c_int8), s.shape[0], _ptr(nn, ctypes.c_int8))
    return nn


def half_sweep(spins: np.ndarray, beta: float, seed: int, t: int, q: int) -> None:
    s = _lattice(spins)
    T = np.array(thresholds(beta), dtype=np.uint64)
    _load().oracle_half_sweep(_ptr(s, ctypes.c_int8), s.shape[0], _ptr(T, ctypes.c_uint64),
                              seed, t, q)


def sweep(spins: np.ndarray, beta: float, n: int, seed: int, offset: int = 0,
          trace: bool = False):
    """Run n sweeps in place; returns the (n, 2) int64 (M, E) trace when ``trace``."""
    s = _lattice(spins)
    tr = np.zeros((max(n, 0), 2), dtype=np.int64) if trace else None
    _load().oracle_sweep(_ptr(s, ctypes.c_int8), s.shape[0], float(beta), n, seed, offset,
                         _ptr(tr, ctypes.c_int64) if tr is not None else None)
    return tr


def observables(spins: np.ndarray) -> tuple[int, int]:
    s = _lattice(spins)
    out = np.zeros(2, dtype=np.int64)
    _load().oracle_observables(_ptr(s, ctypes.c_int8), s.shape[0], _ptr(out, ctypes.c_int64))
    return int(out[0]), int(out[1])


def crop(L: int, seed: int, beta: float, n: int, offset: int, r0: int, c0: int, h: int,
         w: int) -> np.ndarray:
    out = np.empty((h, w), dtype=np.int8)
    _load().oracle_crop(L, seed, float(beta), n, offset, r0, c0, h, w, _ptr(out, ctypes.c_int8))
    return out


FMT = {"bf16": 1, "fp16": 2}


def round_fmt(v: float, fmt: str, toward_zero: bool = False) -> float:
    return float(_load().oracle_round_fmt(float(v), FMT[fmt], int(toward_zero)))


def p_fmt(beta: float, s: int, fmt: str) -> float:
    return float(_load().oracle_p_fmt(float(beta), s, FMT[fmt]))


def u_fmt(x: int, fmt: str) -> float:
    return float(_load().oracle_u_fmt(x, FMT[fmt]))


def sweep_fmt(spins: np.ndarray, beta: float, fmt: str, n: int, seed: int, offset: int = 0,
              trace: bool = False):
    """n sweeps with low-precision acceptance (fmt "bf16" or "fp16")."""
    s = _lattice(spins)
    tr = np.zeros((max(n, 0), 2), dtype=np.int64) if trace else None
    _load().oracle_sweep_fmt(_ptr(s, ctypes.c_int8), s.shape[0], float(beta), FMT[fmt], n, seed, offset,
                             _ptr(tr, ctypes.c_int64) if tr is not None else None)
    return tr


# ---- three dimensions: L x L x L torus, int8 array of shape (L, L, L) indexed [z, y, x]

def _cube(spins: np.ndarray) -> np.ndarray:
    if spins.dtype != np.int8 or spins.ndim != 3 or not (spins.shape[0] == spins.shape[1] == spins.shape[2]):
        raise ValueError("lattice must be a cubic int8 array")
    if not spins.flags.c_contiguous:
        raise ValueError("lattice must be C-contiguous")
    return spins


def thresholds3(beta: float) -> tuple[int, int, int]:
    T = np.zeros(3, dtype=np.uint64)
    _load().oracle3_thresholds(float(beta), _ptr(T, ctypes.c_uint64))
    return int(T[0]), int(T[1]), int(T[2])


def init3(L: int, seed: int) -> np.ndarray:
    s = np.empty((L, L, L), dtype=np.int8)
    _load().oracle3_init(_ptr(s, ctypes.c_int8), L, seed)
    return s


def local_field3(spins: np.ndarray) -> np.ndarray:
    s = _cube(spins)
    nn = np.empty_like(s)
    _load().oracle3_local_field(_ptr(s, ctypes.c_int8), s.shape[0], _ptr(nn, ctypes.c_int8))
    return nn


def half_sweep3(spins: np.ndarray, beta: float, seed: int, t: int, q: int) -> None:
    s = _cube(spins)
    T = np.array(thresholds3(beta), dtype=np.uint64)
    _load().oracle3_half_sweep(_ptr(s, ctypes.c_int8), s.shape[0], _ptr(T, ctypes.c_uint64), seed, t, q)


def sweep3(spins: np.ndarray, beta: float, n: int, seed: int, offset: int = 0, trace: bool = False):
    s = _cube(spins)
    tr = np.zeros((max(n, 0), 2), dtype=np.int64) if trace else None
    _load().oracle3_sweep(_ptr(s, ctypes.c_int8), s.shape[0], float(beta), n, seed, offset,
                          _ptr(tr, ctypes.c_int64) if tr is not None else None)
    return tr


def observables3(spins: np.ndarray) -> tuple[int, int]:
    s = _cube(spins)
    out = np.zeros(2, dtype=np.int64)
    _load().oracle3_observables(_ptr(s, ctypes.c_int8), s.shape[0], _ptr(out, ctypes.c_int64))
    return int(out[0]), int(out[1])


def crop3(L: int, seed: int, beta: float, n: int, offset: int, z0: int, y0: int, x0: int, d: int, h: int,
          w: int) -> np.ndarray:
    out = np.empty((d, h, w), dtype=np.int8)
    _load().oracle3_crop(L, seed, float(beta), n, offset, z0, y0, x0, d, h, w, _ptr(out, ctypes.c_int8))
    return out


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def moments(trace: np.ndarray, n_sites: int) -> np.ndarray:
    """(<|m|>, <m^2>, <m^4>, <e>, <e^2>) of an (n, 2) int64 (M, E) trace, FP64 sums in sweep order."""
    tr = np.ascontiguousarray(trace, dtype=np.int64)
    out = np.zeros(5, dtype=np.float64)
    _load().oracle_moments(_ptr(tr, ctypes.c_int64), tr.shape[0], int(n_sites), _ptr(out, ctypes.c_double))
    return out
