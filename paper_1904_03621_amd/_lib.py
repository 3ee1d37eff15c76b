"""ctypes binding of libsgpu.so (include/sg.h).  Argument marshalling only:
every step of the search runs in the library's HIP kernels.

The functions named ``sg_*`` mirror the C entry points one to one and take
torch tensors that already live on the GPU (the library reads and writes
them through their device pointers, on the current HIP stream).
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgpu.so")

SG_OK, SG_EINVAL, SG_ENONFINITE, SG_EOVERFLOW, SG_ENOMEM, SG_EHIP, \
    SG_EUNSUPPORTED, SG_EDRIFT, SG_ECAPACITY = range(9)
STATUS_NAMES = {
    0: "SG_OK", 1: "SG_EINVAL", 2: "SG_ENONFINITE", 3: "SG_EOVERFLOW", 4: "SG_ENOMEM",
    5: "SG_EHIP", 6: "SG_EUNSUPPORTED", 7: "SG_EDRIFT", 8: "SG_ECAPACITY",
}
SG_MAX_N = 63
SG_MAX_S = 1 << 20
SG_MAX_S_BATCHED = 4096
SG_MAX_DOS_BINS = 8192

# every symbol include/sg.h declares
EXPORTS = [
    "sg_low_spectrum_f32", "sg_low_spectrum_i32",
    "sg_low_spectrum_range_f32", "sg_low_spectrum_range_i32",
    "sg_low_spectrum_batched_f32", "sg_low_spectrum_batched_i32",
    "sg_logz_forward_f32", "sg_logz_backward_f32", "sg_logz_backward_noalloc_f32",
    "sg_reserve",
    "sg_density_of_states_i32", "sg_energy_bound_i32", "sg_tune_batched_f32",
    "sg_low_spectrum_qubo_f32",
    "sg_get_error", "sg_last_error", "sg_get_run_info", "sg_debug_plan",
    "sg_set_kernel_timing", "sg_probe_valu",
    "sg_debug_set_fill", "sg_debug_set_margin_scale", "sg_debug_set_batch_shift",
]
PROBE_OPS = {"v_add_f32": 0, "v_min3_f32": 1, "v_add_u32": 2, "v_min3_i32": 3, "v_fma_f32": 4,
             "v_min_f32": 5, "v_or_b32": 6, "v_or3_b32": 7, "v_add3_u32": 8, "v_max3_f32": 9,
             "v_min_i32": 10, "v_sub_f32": 11, "v_and_or_b32": 12, "v_med3_f32": 13,
             "v_pk_add_u16": 14, "v_pk_min_i16": 15, "v_exp_f32": 16, "v_sub_u32": 17,
             "v_and_b32": 18, "v_cvt_i32_f32": 19, "v_lshl_add_u32": 20,
             # instruction mixes of the walk's steps (lane-instructions/s)
             "mix_f32_walk": 21, "mix_packed_walk": 22, "mix_packed_walk_1chain": 23,
             "mix_packed_walk_2chains": 24, "mix_f32_walk_1chain": 25,
             "mix_packed_walk_1chain_64vgpr": 26, "mix_packed_walk_1chain_long": 27}


class SgError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))


class RunInfo(ctypes.Structure):
    _fields_ = [
        ("chunks", ctypes.c_int64),
        ("candidates", ctypes.c_int64),
        ("slow_blocks", ctypes.c_int64),
        ("margin", ctypes.c_double),
        ("max_drift", ctypes.c_double),
        ("prefix_bits_max", ctypes.c_int32),
        ("free_bits_max", ctypes.c_int32),
        ("enum_launches", ctypes.c_int64),
        ("enum_states", ctypes.c_double),
        ("enum_ms", ctypes.c_double),
        ("max_chunk_candidates", ctypes.c_int64),
        ("repeated_passes", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libsgpu.so is not built (%s); run __graft_entry__.build() or "
                "python paper_1904_03621_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        for name in ("sg_low_spectrum_f32", "sg_low_spectrum_i32"):
            f = getattr(L, name)
            f.restype = i32
            f.argtypes = [i32, vp, vp, i32, vp, vp, vp]
        for name in ("sg_low_spectrum_range_f32", "sg_low_spectrum_range_i32"):
            f = getattr(L, name)
            f.restype = i32
            f.argtypes = [i32, vp, vp, i32, u64, u64, vp, vp, vp]
        for name in ("sg_low_spectrum_batched_f32", "sg_low_spectrum_batched_i32"):
            f = getattr(L, name)
            f.restype = i32
            f.argtypes = [i32, vp, i32, vp, vp, i32, vp, vp, vp]
        L.sg_logz_forward_f32.restype = i32
        L.sg_logz_forward_f32.argtypes = [i32, i32, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp]
        L.sg_logz_backward_f32.restype = i32
        L.sg_logz_backward_f32.argtypes = [i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.sg_logz_backward_noalloc_f32.restype = i32
        L.sg_logz_backward_noalloc_f32.argtypes = [i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                                   vp]
        L.sg_density_of_states_i32.restype = i32
        L.sg_density_of_states_i32.argtypes = [i32, vp, vp, ctypes.c_longlong, i32, vp, vp]
        L.sg_energy_bound_i32.restype = i32
        L.sg_energy_bound_i32.argtypes = [i32, vp, vp, vp, vp]
        L.sg_low_spectrum_qubo_f32.restype = i32
        L.sg_low_spectrum_qubo_f32.argtypes = [i32, vp, vp, i32, vp, vp, vp]
        L.sg_tune_batched_f32.restype = i32
        L.sg_tune_batched_f32.argtypes = [i32, vp, i32, vp, vp, i32, vp, vp]
        L.sg_reserve.restype = i32
        L.sg_reserve.argtypes = [i32, i32, i32, vp]
        L.sg_get_error.restype = i32
        L.sg_get_error.argtypes = [vp]
        L.sg_last_error.restype = ctypes.c_char_p
        L.sg_last_error.argtypes = []
        L.sg_get_run_info.restype = i32
        L.sg_get_run_info.argtypes = [vp, ctypes.POINTER(RunInfo)]
        L.sg_probe_valu.restype = ctypes.c_double
        L.sg_probe_valu.argtypes = [i32, i32]
        L.sg_set_kernel_timing.restype = None
        L.sg_set_kernel_timing.argtypes = [i32]
        L.sg_debug_set_fill.restype = i32
        L.sg_debug_set_fill.argtypes = [vp, ctypes.c_longlong]
        L.sg_debug_set_margin_scale.restype = i32
        L.sg_debug_set_margin_scale.argtypes = [vp, ctypes.c_double]
        L.sg_debug_set_batch_shift.restype = i32
        L.sg_debug_set_batch_shift.argtypes = [i32, i32, i32, i32]
        L.sg_debug_plan.restype = i32
        L.sg_debug_plan.argtypes = [i32, i32, u64, u64, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int64), i32]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().sg_last_error().decode()


def check(status: int, where: str) -> None:
    if status != SG_OK:
        raise SgError(status, where, last_error())


def _ptr(t) -> int:
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(getattr(stream, "cuda_stream", stream) or 0)


def sg_low_spectrum_f32(N, J, h, S, states_out, energies_out, stream=None) -> int:
    return lib().sg_low_spectrum_f32(N, _ptr(J), _ptr(h), S, _ptr(states_out),
                                     _ptr(energies_out), _stream(stream))


def sg_low_spectrum_i32(N, J, h, S, states_out, energies_out, stream=None) -> int:
    return lib().sg_low_spectrum_i32(N, _ptr(J), _ptr(h), S, _ptr(states_out),
                                     _ptr(energies_out), _stream(stream))


def sg_low_spectrum_range_f32(N, J, h, S, lo, hi, states_out, energies_out, stream=None) -> int:
    return lib().sg_low_spectrum_range_f32(N, _ptr(J), _ptr(h), S, lo, hi, _ptr(states_out),
                                           _ptr(energies_out), _stream(stream))


def sg_low_spectrum_range_i32(N, J, h, S, lo, hi, states_out, energies_out, stream=None) -> int:
    return lib().sg_low_spectrum_range_i32(N, _ptr(J), _ptr(h), S, lo, hi, _ptr(states_out),
                                           _ptr(energies_out), _stream(stream))


def sg_low_spectrum_batched_f32(B, N_dev, N_max, J, h, S, states_out, energies_out,
                                stream=None) -> int:
    return lib().sg_low_spectrum_batched_f32(B, _ptr(N_dev), N_max, _ptr(J), _ptr(h), S,
                                             _ptr(states_out), _ptr(energies_out),
                                             _stream(stream))


def sg_low_spectrum_batched_i32(B, N_dev, N_max, J, h, S, states_out, energies_out,
                                stream=None) -> int:
    return lib().sg_low_spectrum_batched_i32(B, _ptr(N_dev), N_max, _ptr(J), _ptr(h), S,
                                             _ptr(states_out), _ptr(energies_out),
                                             _stream(stream))


def sg_logz_forward_f32(B, N, J, h, n_beta, beta, S, logz_out, e0_out, states_out,
                        energies_out, stream=None) -> int:
    return lib().sg_logz_forward_f32(B, N, _ptr(J), _ptr(h), n_beta, _ptr(beta), S,
                                     _ptr(logz_out), _ptr(e0_out), _ptr(states_out),
                                     _ptr(energies_out), _stream(stream))


def sg_logz_backward_f32(B, N, J, h, n_beta, beta, e0, logz, grad_logz, grad_J, grad_h,
                         stream=None) -> int:
    return lib().sg_logz_backward_f32(B, N, _ptr(J), _ptr(h), n_beta, _ptr(beta), _ptr(e0),
                                      _ptr(logz), _ptr(grad_logz), _ptr(grad_J), _ptr(grad_h),
                                      _stream(stream))


def sg_logz_backward_noalloc_f32(B, N, J, h, n_beta, beta, e0, logz, grad_logz, grad_J, grad_h,
                                 stream=None) -> int:
    return lib().sg_logz_backward_noalloc_f32(B, N, _ptr(J), _ptr(h), n_beta, _ptr(beta),
                                              _ptr(e0), _ptr(logz), _ptr(grad_logz),
                                              _ptr(grad_J), _ptr(grad_h), _stream(stream))


def sg_density_of_states_i32(N, J, h, e_min, n_bins, counts_out, stream=None) -> int:
    return lib().sg_density_of_states_i32(N, _ptr(J), _ptr(h), e_min, n_bins, _ptr(counts_out),
                                          _stream(stream))


def sg_energy_bound_i32(N, J, h, bound_out, stream=None) -> int:
    return lib().sg_energy_bound_i32(N, _ptr(J), _ptr(h), _ptr(bound_out), _stream(stream))


def sg_low_spectrum_qubo_f32(N, A, b, S, states_out, energies_out, stream=None) -> int:
    return lib().sg_low_spectrum_qubo_f32(N, _ptr(A), _ptr(b), S, _ptr(states_out),
                                          _ptr(energies_out), _stream(stream))


def sg_tune_batched_f32(B, N_dev, N_max, J, h, S, stream=None) -> int:
    """Runs the tuner; returns the chosen level shift (raises on failure)."""
    out = ctypes.c_int(0)
    st = lib().sg_tune_batched_f32(B, _ptr(N_dev), N_max, _ptr(J), _ptr(h), S,
                                   ctypes.byref(out), _stream(stream))
    check(st, "sg_tune_batched_f32")
    return out.value


def sg_reserve(B_max, N_max, S_max, stream=None) -> int:
    return lib().sg_reserve(B_max, N_max, S_max, _stream(stream))


def sg_get_error(stream=None) -> int:
    return lib().sg_get_error(_stream(stream))


def sg_get_run_info(stream=None) -> dict:
    info = RunInfo()
    check(lib().sg_get_run_info(_stream(stream), ctypes.byref(info)), "sg_get_run_info")
    return info.as_dict()


def sg_set_kernel_timing(enable: bool) -> None:
    lib().sg_set_kernel_timing(1 if enable else 0)


def sg_probe_valu(op, waves_per_simd: int = 8) -> float:
    """Measured lane-instructions/s of one VALU instruction kind (name or code)."""
    code = PROBE_OPS[op] if isinstance(op, str) else int(op)
    return float(lib().sg_probe_valu(code, waves_per_simd))


def sg_debug_set_fill(lanes: int, stream=None) -> int:
    return lib().sg_debug_set_fill(_stream(stream), int(lanes))


def sg_debug_set_margin_scale(scale: float, stream=None) -> int:
    return lib().sg_debug_set_margin_scale(_stream(stream), float(scale))


def sg_debug_set_batch_shift(B: int, N_max: int, S: int, shift: int) -> int:
    return lib().sg_debug_set_batch_shift(B, N_max, S, shift)


def sg_debug_plan(N, S, lo, hi, lanes_fill, cap=100000):
    fm = (ctypes.c_uint64 * cap)()
    nb = (ctypes.c_int32 * cap)()
    ln = (ctypes.c_int64 * cap)()
    k = lib().sg_debug_plan(N, S, lo, hi, lanes_fill, fm, nb, ln, cap)
    if k < 0:
        raise SgError(SG_EINVAL, "sg_debug_plan", "bad arguments")
    k = min(k, cap)
    return [(int(fm[i]), int(nb[i]), int(ln[i])) for i in range(k)]
