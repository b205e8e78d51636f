"""MI355X-native checkerboard Metropolis sweep of the periodic 2D Ising model.

The hot path (arXiv 1903.11714, Sec. 3.1-3.2) runs in hand-written HIP kernels for gfx950
behind the C ABI in include/ising.h; ``paper_1903_11714_amd.ising`` is its ctypes binding.
"""
from . import ising  # noqa: F401
from .ising import (  # noqa: F401
    IsingError,
    batch_run,
    ising_batch_run,
    ising_batch_unpack,
    ising_batch_workspace_bytes,
    ising_fill,
    ising_fill_packed,
    ising_get_option,
    ising_set_option,
    ising_half_sweep,
    ising_half_sweep_packed,
    ising_init_packed,
    ising_moments,
    ising_sweep_fmt,
    ising_sweep_fused,
    ising3_fill,
    ising3_half_sweep,
    ising3_init,
    ising3_observables,
    ising3_sweep,
    ising3_thresholds,
    ising_sweep_fused_step,
    ising_sweep_packed_fmt,
    ising_thresholds_fmt,
    ising_init,
    ising_observables,
    ising_observables_packed,
    ising_pack,
    ising_sweep,
    ising_sweep_packed,
    ising_thresholds,
    ising_unpack,
    ising_version,
    new_lattice,
    new_packed,
    observables,
)
