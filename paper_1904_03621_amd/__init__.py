"""Exhaustive Ising low-spectrum search on AMD MI355X (gfx950).

Implements the exhaustive search of "Brute-forcing spin-glass problems with
CUDA" (arXiv:1904.03621): all 2^N configurations of an Ising instance on an
arbitrary graph are enumerated and the S lowest are returned.  The work runs in
hand-written HIP kernels behind the C ABI of include/sg.h; this package is the
Python binding (ctypes + torch tensors as device buffers).
"""

from .api import (  # noqa: F401
    low_spectrum, low_spectrum_range, low_spectrum_batched, run_info, logz, logz_forward,
    logz_backward, density_of_states, low_spectrum_qubo,
)
from ._lib import (  # noqa: F401
    SgError, sg_low_spectrum_f32, sg_low_spectrum_i32, sg_low_spectrum_range_f32,
    sg_low_spectrum_range_i32, sg_get_error, sg_get_run_info, sg_debug_plan,
    sg_set_kernel_timing, sg_probe_valu, sg_low_spectrum_batched_f32,
    sg_low_spectrum_batched_i32, sg_logz_forward_f32, sg_logz_backward_f32,
    sg_logz_backward_noalloc_f32, sg_reserve, sg_density_of_states_i32, sg_energy_bound_i32, sg_tune_batched_f32,
    sg_low_spectrum_qubo_f32,
)
