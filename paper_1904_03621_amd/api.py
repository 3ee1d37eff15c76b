"""Tensor-level wrappers: allocate the outputs and call the C entry points.

``J`` and ``h`` are torch tensors on the GPU (float32 or int32); ``J`` is
dense N x N of which the strict upper triangle is read.  Masks come back as
int64 tensors (values < 2^56, bit i = spin i, set bit = spin up).
"""

from __future__ import annotations

from . import _lib


def _prep(J, h):
    import torch
    if J.dim() != 2 or J.shape[0] != J.shape[1] or h.dim() != 1 or h.shape[0] != J.shape[0]:
        raise ValueError("J must be N x N and h of length N")
    if not (J.is_cuda and h.is_cuda):
        raise ValueError("J and h must be GPU tensors")
    if J.dtype != h.dtype or J.dtype not in (torch.float32, torch.int32):
        raise ValueError("J and h must both be float32 or both int32")
    return J.contiguous(), h.contiguous()


def low_spectrum_range(J, h, S: int, lo: int, hi: int, stream=None, check: bool = True):
    """S lowest (mask, energy) among masks in [lo, hi), ascending by (E, mask)."""
    import torch
    J, h = _prep(J, h)
    N = J.shape[0]
    states = torch.empty(S, dtype=torch.int64, device=J.device)
    energies = torch.empty(S, dtype=J.dtype, device=J.device)
    if J.dtype == torch.float32:
        st = _lib.sg_low_spectrum_range_f32(N, J, h, S, lo, hi, states, energies, stream)
    else:
        st = _lib.sg_low_spectrum_range_i32(N, J, h, S, lo, hi, states, energies, stream)
    _lib.check(st, "sg_low_spectrum_range")
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return states, energies


def low_spectrum(J, h, S: int, stream=None, check: bool = True):
    """The S lowest states of the instance and their energies (all 2^N searched)."""
    import torch
    J, h = _prep(J, h)
    N = J.shape[0]
    states = torch.empty(S, dtype=torch.int64, device=J.device)
    energies = torch.empty(S, dtype=J.dtype, device=J.device)
    if J.dtype == torch.float32:
        st = _lib.sg_low_spectrum_f32(N, J, h, S, states, energies, stream)
    else:
        st = _lib.sg_low_spectrum_i32(N, J, h, S, states, energies, stream)
    _lib.check(st, "sg_low_spectrum")
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return states, energies


def run_info(stream=None) -> dict:
    return _lib.sg_get_run_info(stream)
