"""Thin ctypes binding of ``libising.so`` (the C ABI declared in include/ising.h).

Argument marshalling only: every step of the sweep runs in the HIP kernels of the library.
PyTorch supplies device memory and the stream.  There is no fallback: if the library is not
built, or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libising.so")

ISING_OK = 0
ISING_EINVAL = -1
ISING_EHIP = -2
ISING_EUNSUPPORTED = -3

_lib = None


class IsingError(RuntimeError):
    def __init__(self, func: str, status: int, detail: str = ""):
        self.status = status
        msg = f"{func} failed with status {status}"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class ReplicaT(ctypes.Structure):
    """ising_replica_t: one lattice of a batch."""
    _fields_ = [("L", ctypes.c_int64), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64)]


_SIGNATURES = {
    "ising_init": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p], ctypes.c_int),
    "ising_fill": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising_sweep": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_half_sweep": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising_observables": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_pack": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_unpack": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_sweep_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_observables_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
                                 ctypes.c_int),
    "ising_init_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p], ctypes.c_int),
    "ising_fill_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising_packed_words": ([ctypes.c_int64], ctypes.c_int64),
    "ising_half_sweep_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising_thresholds": ([ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "ising_thresholds_fmt": ([ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "ising_sweep_fmt": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                         ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_sweep_packed_fmt": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_sweep_fused": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                           ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p],
                          ctypes.c_int),
    "ising_sweep_fused_static": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_sweep_fused_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_sweep_fused_pair": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_init": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p], ctypes.c_int),
    "ising3_fill": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising3_sweep": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                      ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_sweep_fused": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_sweep_fused_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_half_sweep": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                           ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising3_observables": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_thresholds": ([ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "ising3_pack": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_unpack": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_init_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p], ctypes.c_int),
    "ising3_sweep_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                             ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising3_half_sweep_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ising3_observables_packed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_moments": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
                      ctypes.c_int),
    "ising_batch_workspace_bytes": ([ctypes.POINTER(ReplicaT), ctypes.c_int64], ctypes.c_int64),
    "ising_batch_run": ([ctypes.POINTER(ReplicaT), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ising_batch_schedule": ([ctypes.POINTER(ReplicaT), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ising_batch_unpack": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
                           ctypes.c_int),
    "ising_set_option": ([ctypes.c_char_p, ctypes.c_int64], ctypes.c_int),
    "ising_get_option": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ising_last_error": ([], ctypes.c_char_p),
    "ising_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "ising_version": ([], ctypes.c_int),
}


def library():
    """Load libising.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1903_11714_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(name: str, status: int) -> None:
    if status != ISING_OK:
        lib = library()
        detail = lib.ising_strerror(status).decode()
        if status == ISING_EHIP:
            detail += " (" + lib.ising_last_error().decode() + ")"
        raise IsingError(name, status, detail)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype_name: str, numel: int | None = None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) tensor")
    if str(t.dtype) != dtype_name:
        raise TypeError(f"expected dtype {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _opt_ptr(t, dtype_name: str, numel: int):
    return None if t is None else _dev_ptr(t, dtype_name, numel)


def _packed_n(L: int):
    """Words of the packed layout for L (None for an invalid L: the library call then rejects it)."""
    n = library().ising_packed_words(L)
    return n if n >= 0 else None


def ising_packed_words(L: int) -> int:
    """uint32 words of both colour planes of an L x L lattice: 2 L ceil(L / 64)."""
    n = library().ising_packed_words(L)
    if n < 0:
        _check("ising_packed_words", int(n))
    return int(n)


# ---- same names as the C ABI -----------------------------------------------------------------

def ising_init(spins, L: int, seed: int, stream=None) -> None:
    _check("ising_init", library().ising_init(_dev_ptr(spins, "torch.int8", L * L), L, seed, _stream(stream)))


def ising_fill(spins, L: int, value: int, stream=None) -> None:
    _check("ising_fill", library().ising_fill(_dev_ptr(spins, "torch.int8", L * L), L, value, _stream(stream)))


def ising_sweep(spins, L: int, beta: float, n_sweeps: int, seed: int, sweep_offset: int = 0,
                trace_ME=None, stream=None) -> None:
    _check("ising_sweep", library().ising_sweep(
        _dev_ptr(spins, "torch.int8", L * L), L, float(beta), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising_half_sweep(spins, L: int, beta: float, seed: int, t: int, q: int, stream=None) -> None:
    _check("ising_half_sweep", library().ising_half_sweep(
        _dev_ptr(spins, "torch.int8", L * L), L, float(beta), seed, t, q, _stream(stream)))


def ising_observables(spins, L: int, out_ME, stream=None) -> None:
    _check("ising_observables", library().ising_observables(
        _dev_ptr(spins, "torch.int8", L * L), L, _dev_ptr(out_ME, "torch.int64", 2), _stream(stream)))


def ising_pack(spins, L: int, planes, stream=None) -> None:
    _check("ising_pack", library().ising_pack(
        _dev_ptr(spins, "torch.int8", L * L), L, _dev_ptr(planes, "torch.int32", _packed_n(L)), _stream(stream)))


def ising_unpack(planes, L: int, spins, stream=None) -> None:
    _check("ising_unpack", library().ising_unpack(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, _dev_ptr(spins, "torch.int8", L * L), _stream(stream)))


def ising_sweep_packed(planes, L: int, beta: float, n_sweeps: int, seed: int, sweep_offset: int = 0,
                       trace_ME=None, stream=None) -> None:
    _check("ising_sweep_packed", library().ising_sweep_packed(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, float(beta), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising_init_packed(planes, L: int, seed: int, stream=None) -> None:
    _check("ising_init_packed", library().ising_init_packed(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, seed, _stream(stream)))


def ising_fill_packed(planes, L: int, value: int, stream=None) -> None:
    _check("ising_fill_packed", library().ising_fill_packed(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, value, _stream(stream)))


def ising_half_sweep_packed(planes, L: int, beta: float, seed: int, t: int, q: int, stream=None) -> None:
    _check("ising_half_sweep_packed", library().ising_half_sweep_packed(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, float(beta), seed, t, q, _stream(stream)))


def ising_observables_packed(planes, L: int, out_ME, stream=None) -> None:
    _check("ising_observables_packed", library().ising_observables_packed(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, _dev_ptr(out_ME, "torch.int64", 2), _stream(stream)))


def ising_thresholds(beta: float) -> tuple[int, int]:
    out = (ctypes.c_uint64 * 2)()
    _check("ising_thresholds", library().ising_thresholds(float(beta), out))
    return int(out[0]), int(out[1])


FMT = {"exact": 0, "bf16": 1, "fp16": 2}


def _fmt(fmt) -> int:
    return FMT[fmt] if isinstance(fmt, str) else int(fmt)


def ising_thresholds_fmt(beta: float, fmt) -> tuple[int, int]:
    out = (ctypes.c_uint64 * 2)()
    _check("ising_thresholds_fmt", library().ising_thresholds_fmt(float(beta), _fmt(fmt), out))
    return int(out[0]), int(out[1])


def ising_sweep_fmt(spins, L: int, beta: float, fmt, n_sweeps: int, seed: int, sweep_offset: int = 0,
                    trace_ME=None, stream=None) -> None:
    _check("ising_sweep_fmt", library().ising_sweep_fmt(
        _dev_ptr(spins, "torch.int8", L * L), L, float(beta), _fmt(fmt), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising_sweep_fused(spins, scratch, L: int, beta: float, fmt, n_sweeps: int, seed: int, sweep_offset: int = 0,
                      trace_ME=None, stream=None) -> None:
    _check("ising_sweep_fused", library().ising_sweep_fused(
        _dev_ptr(spins, "torch.int8", L * L), _dev_ptr(scratch, "torch.int8", L * L), L, float(beta), _fmt(fmt),
        n_sweeps, seed, sweep_offset, _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising_sweep_fused_static(spins, L: int, beta: float, fmt, n_sweeps: int, seed: int, sweep_offset: int = 0,
                             trace_ME=None, stream=None) -> None:
    _check("ising_sweep_fused_static", library().ising_sweep_fused_static(
        _dev_ptr(spins, "torch.int8", L * L), L, float(beta), _fmt(fmt), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising_sweep_fused_step(src, dst, L: int, beta: float, fmt, seed: int, t: int, out_ME=None,
                           stream=None) -> None:
    _check("ising_sweep_fused_step", library().ising_sweep_fused_step(
        _dev_ptr(src, "torch.int8", L * L), _dev_ptr(dst, "torch.int8", L * L), L, float(beta), _fmt(fmt), seed, t,
        _opt_ptr(out_ME, "torch.int64", 2), _stream(stream)))


def ising_sweep_fused_pair(src, dst, L: int, beta: float, fmt, seed: int, t: int, out_ME=None,
                           stream=None) -> None:
    _check("ising_sweep_fused_pair", library().ising_sweep_fused_pair(
        _dev_ptr(src, "torch.int8", L * L), _dev_ptr(dst, "torch.int8", L * L), L, float(beta), _fmt(fmt), seed, t,
        _opt_ptr(out_ME, "torch.int64", 4), _stream(stream)))


def ising3_init(spins, L: int, seed: int, stream=None) -> None:
    _check("ising3_init", library().ising3_init(_dev_ptr(spins, "torch.int8", L ** 3), L, seed, _stream(stream)))


def ising3_fill(spins, L: int, value: int, stream=None) -> None:
    _check("ising3_fill", library().ising3_fill(_dev_ptr(spins, "torch.int8", L ** 3), L, value, _stream(stream)))


def ising3_sweep(spins, L: int, beta: float, n_sweeps: int, seed: int, sweep_offset: int = 0, trace_ME=None,
                 stream=None) -> None:
    _check("ising3_sweep", library().ising3_sweep(
        _dev_ptr(spins, "torch.int8", L ** 3), L, float(beta), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising3_sweep_fused(spins, scratch, L: int, beta: float, n_sweeps: int, seed: int, sweep_offset: int = 0,
                       trace_ME=None, stream=None) -> None:
    _check("ising3_sweep_fused", library().ising3_sweep_fused(
        _dev_ptr(spins, "torch.int8", L ** 3), _dev_ptr(scratch, "torch.int8", L ** 3), L, float(beta), n_sweeps,
        seed, sweep_offset, _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising3_sweep_fused_step(src, dst, L: int, beta: float, seed: int, t: int, out_ME=None, stream=None) -> None:
    _check("ising3_sweep_fused_step", library().ising3_sweep_fused_step(
        _dev_ptr(src, "torch.int8", L ** 3), _dev_ptr(dst, "torch.int8", L ** 3), L, float(beta), seed, t,
        _opt_ptr(out_ME, "torch.int64", 2), _stream(stream)))


def ising3_half_sweep(spins, L: int, beta: float, seed: int, t: int, q: int, stream=None) -> None:
    _check("ising3_half_sweep", library().ising3_half_sweep(
        _dev_ptr(spins, "torch.int8", L ** 3), L, float(beta), seed, t, q, _stream(stream)))


def ising3_observables(spins, L: int, out_ME, stream=None) -> None:
    _check("ising3_observables", library().ising3_observables(
        _dev_ptr(spins, "torch.int8", L ** 3), L, _dev_ptr(out_ME, "torch.int64", 2), _stream(stream)))


def ising3_thresholds(beta: float) -> tuple[int, int, int]:
    out = (ctypes.c_uint64 * 3)()
    _check("ising3_thresholds", library().ising3_thresholds(float(beta), out))
    return int(out[0]), int(out[1]), int(out[2])


def ising3_pack(spins, L: int, planes, stream=None) -> None:
    _check("ising3_pack", library().ising3_pack(
        _dev_ptr(spins, "torch.int8", L ** 3), L, _dev_ptr(planes, "torch.int32", L ** 3 // 32), _stream(stream)))


def ising3_unpack(planes, L: int, spins, stream=None) -> None:
    _check("ising3_unpack", library().ising3_unpack(
        _dev_ptr(planes, "torch.int32", L ** 3 // 32), L, _dev_ptr(spins, "torch.int8", L ** 3), _stream(stream)))


def ising3_init_packed(planes, L: int, seed: int, stream=None) -> None:
    _check("ising3_init_packed", library().ising3_init_packed(
        _dev_ptr(planes, "torch.int32", L ** 3 // 32), L, seed, _stream(stream)))


def ising3_sweep_packed(planes, L: int, beta: float, n_sweeps: int, seed: int, sweep_offset: int = 0,
                        trace_ME=None, stream=None) -> None:
    _check("ising3_sweep_packed", library().ising3_sweep_packed(
        _dev_ptr(planes, "torch.int32", L ** 3 // 32), L, float(beta), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising3_half_sweep_packed(planes, L: int, beta: float, seed: int, t: int, q: int, stream=None) -> None:
    _check("ising3_half_sweep_packed", library().ising3_half_sweep_packed(
        _dev_ptr(planes, "torch.int32", L ** 3 // 32), L, float(beta), seed, t, q, _stream(stream)))


def ising3_observables_packed(planes, L: int, out_ME, stream=None) -> None:
    _check("ising3_observables_packed", library().ising3_observables_packed(
        _dev_ptr(planes, "torch.int32", L ** 3 // 32), L, _dev_ptr(out_ME, "torch.int64", 2), _stream(stream)))


def ising_sweep_packed_fmt(planes, L: int, beta: float, fmt, n_sweeps: int, seed: int, sweep_offset: int = 0,
                           trace_ME=None, stream=None) -> None:
    _check("ising_sweep_packed_fmt", library().ising_sweep_packed_fmt(
        _dev_ptr(planes, "torch.int32", _packed_n(L)), L, float(beta), _fmt(fmt), n_sweeps, seed, sweep_offset,
        _opt_ptr(trace_ME, "torch.int64", 2 * n_sweeps), _stream(stream)))


def ising_moments(trace_ME, n: int, n_sites: int, out, stream=None) -> None:
    _check("ising_moments", library().ising_moments(
        _dev_ptr(trace_ME, "torch.int64", 2 * n), n, n_sites, _dev_ptr(out, "torch.float64", 5), _stream(stream)))


def _replica_array(replicas):
    arr = (ReplicaT * len(replicas))()
    for i, (L, beta, seed) in enumerate(replicas):
        arr[i] = ReplicaT(int(L), float(beta), int(seed))
    return arr


def ising_batch_workspace_bytes(replicas) -> int:
    """replicas: sequence of (L, beta, seed)."""
    n = int(library().ising_batch_workspace_bytes(_replica_array(replicas), len(replicas)))
    if n < 0:
        raise IsingError("ising_batch_workspace_bytes", n, "invalid replica table")
    return n


def ising_batch_run(replicas, n_therm: int, n_meas: int, workspace, sweep_offset: int = 0, fmt=0, start: int = 0,
                    trace_ME=None, moments=None, stream=None) -> None:
    n = len(replicas)
    _check("ising_batch_run", library().ising_batch_run(
        _replica_array(replicas), n, n_therm, n_meas, sweep_offset, _fmt(fmt), start,
        _dev_ptr(workspace, "torch.uint8"), workspace.numel(),
        _opt_ptr(trace_ME, "torch.int64", 2 * n * n_meas), _opt_ptr(moments, "torch.float64", 5 * n),
        _stream(stream)))


def ising_batch_schedule(replicas) -> tuple[int, int, int, int]:
    """(threads per workgroup, split target in sites per slab or -1, colour updates between
    exchanges, work lists per compute unit) that ising_batch_run tuned for this set of replica
    sizes."""
    out = (ctypes.c_int64 * 4)()
    _check("ising_batch_schedule", library().ising_batch_schedule(_replica_array(replicas), len(replicas), out))
    return int(out[0]), int(out[1]), int(out[2]), int(out[3])


def ising_batch_unpack(workspace, n: int, j: int, spins, stream=None) -> None:
    _check("ising_batch_unpack", library().ising_batch_unpack(
        _dev_ptr(workspace, "torch.uint8"), n, j, _dev_ptr(spins, "torch.int8"), _stream(stream)))


def ising_set_option(name: str, value: int) -> None:
    _check("ising_set_option", library().ising_set_option(name.encode(), int(value)))


def ising_get_option(name: str) -> int:
    v = ctypes.c_int64()
    _check("ising_get_option", library().ising_get_option(name.encode(), ctypes.byref(v)))
    return int(v.value)


def ising_version() -> int:
    return int(library().ising_version())


# ---- conveniences built only from the calls above ---------------------------------------------

def new_lattice(L: int, seed: int | None = None, device: str = "cuda"):
    """Allocate an L x L int8 lattice; hot start from `seed`, or all +1 when seed is None."""
    import torch
    spins = torch.empty((L, L), dtype=torch.int8, device=device)
    if seed is None:
        ising_fill(spins, L, 1)
    else:
        ising_init(spins, L, seed)
    return spins


def new_packed(L: int, seed: int | None, device: str = "cuda"):
    """Allocate the packed form of an L x L lattice (int32 words): hot start of `seed`, or all +1
    when seed is None."""
    import torch
    planes = torch.empty(_packed_n(L), dtype=torch.int32, device=device)
    if seed is None:
        ising_fill_packed(planes, L, 1)
    else:
        ising_init_packed(planes, L, seed)
    return planes


def batch_run(replicas, n_therm: int, n_meas: int, fmt=0, start: int = 0, sweep_offset: int = 0,
              trace: bool = True, workspace=None, device: str = "cuda"):
    """Run a batch of (L, beta, seed) replicas in one persistent launch.  Returns
    (moments [n, 5] float64: <|m|>, <m^2>, <m^4>, <e>, <e^2>; trace [n, n_meas, 2] int64 or None;
    workspace, which holds the lattices for a later start=2 call)."""
    import torch
    n = len(replicas)
    if workspace is None:
        workspace = torch.empty(ising_batch_workspace_bytes(replicas), dtype=torch.uint8, device=device)
    moments = torch.empty((n, 5), dtype=torch.float64, device=device)
    tr = torch.empty((n, max(n_meas, 1), 2), dtype=torch.int64, device=device) if trace and n_meas else None
    ising_batch_run(replicas, n_therm, n_meas, workspace, sweep_offset, fmt, start,
                    tr.view(-1)[: 2 * n * n_meas] if tr is not None else None, moments)
    return moments, tr, workspace


def observables(spins) -> tuple[int, int]:
    """(M, E) of an int8 lattice; synchronises to read the result."""
    import torch
    L = spins.shape[-1]
    out = torch.empty(2, dtype=torch.int64, device=spins.device)
    ising_observables(spins, L, out)
    M, E = out.tolist()
    return int(M), int(E)
