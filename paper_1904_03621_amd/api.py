"""Tensor-level wrappers: allocate the outputs and call the C entry points.

``J`` and ``h`` are torch tensors on the GPU (float32 or int32); ``J`` is
dense N x N of which the strict upper triangle is read.  Masks come back as
int64 tensors (values < 2^63, bit i = spin i, set bit = spin up).
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


def low_spectrum_batched(Ns, J, h, S: int, stream=None, check: bool = True):
    """S lowest states of each of B instances: Ns int32[B] (GPU), J [B, Nmax, Nmax],
    h [B, Nmax] (float32 or int32, GPU).  Returns masks int64[B, S], energies [B, S]."""
    import torch
    if J.dim() != 3 or J.shape[1] != J.shape[2] or h.shape != J.shape[:2]:
        raise ValueError("J must be B x Nmax x Nmax and h B x Nmax")
    if Ns.dtype != torch.int32 or Ns.shape[0] != J.shape[0]:
        raise ValueError("Ns must be int32 of length B")
    if not (J.is_cuda and h.is_cuda and Ns.is_cuda):
        raise ValueError("Ns, J and h must be GPU tensors")
    if J.dtype != h.dtype or J.dtype not in (torch.float32, torch.int32):
        raise ValueError("J and h must both be float32 or both int32")
    J, h, Ns = J.contiguous(), h.contiguous(), Ns.contiguous()
    B, Nmax = J.shape[0], J.shape[1]
    states = torch.empty((B, S), dtype=torch.int64, device=J.device)
    energies = torch.empty((B, S), dtype=J.dtype, device=J.device)
    if J.dtype == torch.float32:
        st = _lib.sg_low_spectrum_batched_f32(B, Ns, Nmax, J, h, S, states, energies, stream)
    else:
        st = _lib.sg_low_spectrum_batched_i32(B, Ns, Nmax, J, h, S, states, energies, stream)
    _lib.check(st, "sg_low_spectrum_batched")
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return states, energies


def _prep_logz(J, h, beta):
    import torch
    if J.dim() != 3 or J.shape[1] != J.shape[2] or h.shape != J.shape[:2]:
        raise ValueError("J must be B x N x N and h B x N")
    if not (J.is_cuda and h.is_cuda and beta.is_cuda):
        raise ValueError("J, h and beta must be GPU tensors")
    if J.dtype != torch.float32 or h.dtype != torch.float32 or beta.dtype != torch.float32:
        raise ValueError("J, h and beta must be float32")
    if beta.dim() != 1:
        raise ValueError("beta must be 1-D")
    return J.contiguous(), h.contiguous(), beta.contiguous()


def logz_forward(J, h, beta, S: int, stream=None, check: bool = True):
    """log Z_b(beta_k) of B instances (J [B, N, N], h [B, N], beta [K], float32,
    GPU).  Returns logz float64[B, K], e0 float32[B], states int64[B, S] and
    energies float32[B, S] (the S lowest states)."""
    import torch
    J, h, beta = _prep_logz(J, h, beta)
    B, N, K = J.shape[0], J.shape[1], beta.shape[0]
    dev = J.device
    logz = torch.empty((B, K), dtype=torch.float64, device=dev)
    e0 = torch.empty(B, dtype=torch.float32, device=dev)
    states = torch.empty((B, S), dtype=torch.int64, device=dev)
    energies = torch.empty((B, S), dtype=torch.float32, device=dev)
    st = _lib.sg_logz_forward_f32(B, N, J, h, K, beta, S, logz, e0, states, energies, stream)
    _lib.check(st, "sg_logz_forward_f32")
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return logz, e0, states, energies


def logz_backward(J, h, beta, e0, logz, grad_logz, stream=None, check: bool = True,
                  no_alloc: bool = False):
    """Gradients (grad_J [B, N, N], upper triangle; grad_h [B, N]) of
    sum grad_logz * logz with respect to J and h.  no_alloc: take the entry
    point whose buffers live in the library's static device scratch (it
    allocates no device memory; limited in B and N)."""
    import torch
    J, h, beta = _prep_logz(J, h, beta)
    B, N, K = J.shape[0], J.shape[1], beta.shape[0]
    if logz.shape != (B, K) or grad_logz.shape != (B, K) or e0.shape != (B,):
        raise ValueError("e0 must be [B], logz and grad_logz [B, K]")
    logz = logz.to(torch.float64).contiguous()
    grad_logz = grad_logz.to(torch.float64).contiguous()
    e0 = e0.to(torch.float32).contiguous()
    gJ = torch.empty((B, N, N), dtype=torch.float32, device=J.device)
    gh = torch.empty((B, N), dtype=torch.float32, device=J.device)
    fn = _lib.sg_logz_backward_noalloc_f32 if no_alloc else _lib.sg_logz_backward_f32
    st = fn(B, N, J, h, K, beta, e0, logz, grad_logz, gJ, gh, stream)
    _lib.check(st, fn.__name__)
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return gJ, gh


def _logz_function():
    import torch

    class LogZ(torch.autograd.Function):
        """log Z(beta) of a batch with exact gradients w.r.t. J and h; the
        backward walks the enumeration again instead of storing weights."""

        @staticmethod
        def forward(ctx, J, h, beta, S):
            logz, e0, states, energies = logz_forward(J, h, beta, S)
            ctx.save_for_backward(J, h, beta, e0, logz)
            ctx.mark_non_differentiable(states, energies)
            return logz, states, energies

        @staticmethod
        def backward(ctx, g_logz, g_states, g_energies):
            J, h, beta, e0, logz = ctx.saved_tensors
            gJ = gh = None
            if g_logz is not None and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]):
                gJ, gh = logz_backward(J, h, beta, e0, logz, g_logz)
            return gJ, gh, None, None

    return LogZ


_LOGZ = None


def logz(J, h, beta, S: int = 32):
    """Differentiable log Z: returns (logz float64[B, K], states int64[B, S],
    energies float32[B, S]); gradients flow to J (upper triangle) and h."""
    global _LOGZ
    if _LOGZ is None:
        _LOGZ = _logz_function()
    return _LOGZ.apply(J, h, beta, S)


def low_spectrum_qubo(A, b, S: int, stream=None, check: bool = True):
    """S lowest binary vectors of the QUBO F(q) = -sum_{i<j} a_ij q_i q_j -
    sum_i b_i q_i (A [N, N] upper triangle, b [N], float32, GPU): returns masks
    int64[S] (bit i = q_i) and F float32[S], ascending by (F, mask)."""
    import torch
    A, b = _prep(A, b)
    if A.dtype != torch.float32:
        raise ValueError("the QUBO front end takes float32 A and b")
    N = A.shape[0]
    states = torch.empty(S, dtype=torch.int64, device=A.device)
    energies = torch.empty(S, dtype=torch.float32, device=A.device)
    _lib.check(_lib.sg_low_spectrum_qubo_f32(N, A, b, S, states, energies, stream),
               "sg_low_spectrum_qubo_f32")
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return states, energies


def density_of_states(J, h, e_min=None, n_bins=None, stream=None, check: bool = True):
    """Exact density of states of an int32 instance (J [N, N], h [N], GPU):
    returns (e_min, counts int64[n_bins]) with counts[k] the number of
    configurations at energy e_min + k.  By default the bins span [-B, B],
    B = sum|J_ij| (i<j) + sum|h_i|, computed on the device."""
    import torch
    J, h = _prep(J, h)
    if J.dtype != torch.int32:
        raise ValueError("the density of states needs int32 J and h")
    N = J.shape[0]
    if e_min is None:
        bound = torch.empty(1, dtype=torch.int64, device=J.device)
        _lib.check(_lib.sg_energy_bound_i32(N, J, h, bound, stream), "sg_energy_bound_i32")
        B = int(bound.item())
        e_min, n_bins = -B, 2 * B + 1
    counts = torch.empty(n_bins, dtype=torch.int64, device=J.device)
    st = _lib.sg_density_of_states_i32(N, J, h, int(e_min), int(n_bins), counts, stream)
    _lib.check(st, "sg_density_of_states_i32")
    if check:
        _lib.check(_lib.sg_get_error(stream), "device")
    return int(e_min), counts


def run_info(stream=None) -> dict:
    return _lib.sg_get_run_info(stream)
