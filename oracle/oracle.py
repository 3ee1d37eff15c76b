"""ctypes binding of the CPU oracle (oracle.c).  TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
module.  It never touches the GPU library and the GPU library never touches it.
"""

from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_u64p = ctypes.POINTER(ctypes.c_uint64)
_c_dp = ctypes.POINTER(ctypes.c_double)
_c_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (portable flags, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load(path: str):
    L = ctypes.CDLL(path)
    L.oracle_max_threads.restype = ctypes.c_int
    L.oracle_max_threads.argtypes = []
    L.oracle_energy_f64.restype = ctypes.c_double
    L.oracle_energy_f64.argtypes = [ctypes.c_int, _c_dp, _c_dp, ctypes.c_uint64]
    L.oracle_energy_i64.restype = ctypes.c_int64
    L.oracle_energy_i64.argtypes = [ctypes.c_int, _c_i64p, _c_i64p, ctypes.c_uint64]
    L.oracle_qubo_from_ising.restype = None
    L.oracle_qubo_from_ising.argtypes = [ctypes.c_int, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp]
    L.oracle_qubo_energy_f64.restype = ctypes.c_double
    L.oracle_qubo_energy_f64.argtypes = [ctypes.c_int, _c_dp, _c_dp, ctypes.c_uint64]
    L.oracle_low_spectrum_f64.restype = ctypes.c_int
    L.oracle_low_spectrum_f64.argtypes = [ctypes.c_int, _c_dp, _c_dp, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_uint64, _c_u64p,
                                          _c_dp, ctypes.c_int]
    L.oracle_low_spectrum_i64.restype = ctypes.c_int
    L.oracle_low_spectrum_i64.argtypes = [ctypes.c_int, _c_i64p, _c_i64p, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_uint64, _c_u64p,
                                          _c_i64p, ctypes.c_int]
    L.oracle_dos_i64.restype = ctypes.c_int
    L.oracle_dos_i64.argtypes = [ctypes.c_int, _c_i64p, _c_i64p, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_uint64, _c_u64p, ctypes.c_int]
    L.oracle_logz_f64.restype = ctypes.c_int
    L.oracle_logz_f64.argtypes = [ctypes.c_int, _c_dp, _c_dp, ctypes.c_int, _c_dp,
                                  _c_dp, _c_dp, _c_dp, _c_dp, ctypes.c_int]
    L.oracle_logz_grad_f64.restype = ctypes.c_int
    L.oracle_logz_grad_f64.argtypes = [ctypes.c_int, _c_dp, _c_dp, ctypes.c_int, _c_dp,
                                       _c_dp, _c_dp, _c_dp, ctypes.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _load(_LIB)
    return _lib


@contextlib.contextmanager
def swapped_library(path: str):
    """Temporarily route every wrapper through another build of oracle.c
    (used by the mutation test, which compiles copies with planted mistakes)."""
    global _lib
    old = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = old


def max_threads() -> int:
    """Threads the oracle's parallel loops use by default."""
    return int(lib().oracle_max_threads())


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _ptr(a, t):
    return a.ctypes.data_as(t)


def is_integer_instance(J, h) -> bool:
    return np.issubdtype(np.asarray(J).dtype, np.integer) and \
        np.issubdtype(np.asarray(h).dtype, np.integer)


def energy(J, h, mask: int):
    """Eq. (1) energy of one state (int for integer instances, float otherwise)."""
    N = len(h)
    if is_integer_instance(J, h):
        Ja, ha = _i64(J), _i64(h)
        return int(lib().oracle_energy_i64(N, _ptr(Ja, _c_i64p), _ptr(ha, _c_i64p), int(mask)))
    Ja, ha = _f64(J), _f64(h)
    return float(lib().oracle_energy_f64(N, _ptr(Ja, _c_dp), _ptr(ha, _c_dp), int(mask)))


def energies(J, h, masks):
    return np.array([energy(J, h, int(m)) for m in masks])


def qubo_from_ising(J, h):
    """Eq. (3): (a, b, offset) with H(s) = F(q) + offset."""
    N = len(h)
    Ja, ha = _f64(J), _f64(h)
    a = np.zeros((N, N)); b = np.zeros(N); off = ctypes.c_double(0.0)
    lib().oracle_qubo_from_ising(N, _ptr(Ja, _c_dp), _ptr(ha, _c_dp), _ptr(a, _c_dp),
                                 _ptr(b, _c_dp), ctypes.byref(off))
    return a, b, off.value


def qubo_energy(a, b, mask: int) -> float:
    """Eq. (2) QUBO cost of one binary vector q (bit i of mask)."""
    aa, bb = _f64(a), _f64(b)
    return float(lib().oracle_qubo_energy_f64(len(bb), _ptr(aa, _c_dp), _ptr(bb, _c_dp), int(mask)))


def low_spectrum(J, h, S: int, lo: int = 0, hi: int | None = None, nthreads: int = 0):
    """The S lowest (E, mask) over masks in [lo, hi), ascending by (E, mask).

    Returns (masks uint64[k], energies[k]) with k = min(S, hi - lo); energies
    are int64 for integer instances and float64 otherwise.
    """
    N = len(h)
    if hi is None:
        hi = 1 << N
    k = max(0, min(S, hi - lo))
    masks = np.zeros(max(k, 1), dtype=np.uint64)
    if is_integer_instance(J, h):
        Ja, ha = _i64(J), _i64(h)
        es = np.zeros(max(k, 1), dtype=np.int64)
        n = lib().oracle_low_spectrum_i64(N, _ptr(Ja, _c_i64p), _ptr(ha, _c_i64p), S, lo, hi,
                                          _ptr(masks, _c_u64p), _ptr(es, _c_i64p), nthreads)
    else:
        Ja, ha = _f64(J), _f64(h)
        es = np.zeros(max(k, 1), dtype=np.float64)
        n = lib().oracle_low_spectrum_f64(N, _ptr(Ja, _c_dp), _ptr(ha, _c_dp), S, lo, hi,
                                          _ptr(masks, _c_u64p), _ptr(es, _c_dp), nthreads)
    return masks[:n], es[:n]


def energy_bound(J, h) -> int:
    """sum_{i<j} |J_ij| + sum_i |h_i| of an integer instance: |E| never exceeds it."""
    N = len(h)
    Ja, ha = _i64(J), _i64(h)
    return int(np.abs(np.triu(Ja.reshape(N, N), 1)).sum() + np.abs(ha).sum())


def density_of_states(J, h, e_min: int | None = None, n_bins: int | None = None,
                      lo: int = 0, hi: int | None = None, nthreads: int = 0):
    """(e_min, counts) with counts[k] the number of masks in [lo, hi) whose
    energy is e_min + k.  By default the bins span [-B, B], B = energy_bound."""
    N = len(h)
    if hi is None:
        hi = 1 << N
    if e_min is None:
        bnd = energy_bound(J, h)
        e_min, n_bins = -bnd, 2 * bnd + 1
    Ja, ha = _i64(J), _i64(h)
    counts = np.zeros(n_bins, dtype=np.uint64)
    rc = lib().oracle_dos_i64(N, _ptr(Ja, _c_i64p), _ptr(ha, _c_i64p), e_min, n_bins, lo, hi,
                              _ptr(counts, _c_u64p), nthreads)
    if rc != 0:
        raise ValueError("an energy falls outside the bins")
    return e_min, counts


def logz(J, h, betas, moments: bool = False, nthreads: int = 0):
    """Exact log Z(beta) for each beta; with moments=True also <s_i>, <s_i s_j>.

    Returns (logz[nb], e0) or (logz[nb], e0, mean_s[nb,N], mean_ss[nb,N,N]).
    """
    N = len(h)
    Ja, ha = _f64(J), _f64(h)
    bt = _f64(np.atleast_1d(betas))
    nb = len(bt)
    lz = np.zeros(nb); e0 = ctypes.c_double(0.0)
    ms = np.zeros((nb, N)) if moments else None
    mss = np.zeros((nb, N, N)) if moments else None
    rc = lib().oracle_logz_f64(N, _ptr(Ja, _c_dp), _ptr(ha, _c_dp), nb, _ptr(bt, _c_dp),
                               _ptr(lz, _c_dp), ctypes.byref(e0),
                               _ptr(ms, _c_dp) if moments else None,
                               _ptr(mss, _c_dp) if moments else None, nthreads)
    if rc != 0:
        raise ValueError("oracle_logz_f64 rejected its arguments")
    if moments:
        return lz, e0.value, ms, mss
    return lz, e0.value


def logz_grad(J, h, betas, g=None, nthreads: int = 0):
    """(grad_J[N,N] upper triangle, grad_h[N]) of sum_b g_b log Z(beta_b)."""
    N = len(h)
    Ja, ha = _f64(J), _f64(h)
    bt = _f64(np.atleast_1d(betas))
    gg = _f64(np.ones(len(bt)) if g is None else np.atleast_1d(g))
    gJ = np.zeros((N, N)); gh = np.zeros(N)
    rc = lib().oracle_logz_grad_f64(N, _ptr(Ja, _c_dp), _ptr(ha, _c_dp), len(bt), _ptr(bt, _c_dp),
                                    _ptr(gg, _c_dp), _ptr(gJ, _c_dp), _ptr(gh, _c_dp), nthreads)
    if rc != 0:
        raise ValueError("oracle_logz_grad_f64 rejected its arguments")
    return gJ, gh
