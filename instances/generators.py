"""Generators of the benchmark and test instances (numbers only).

The paper benchmarks randomly generated fully connected instances (Section 5.1)
whose files are not published with it; the generators below stand in for
them, with the shapes and distributions of the workloads measured here:

* ``random_int_dense``   fully connected, J_ij and h_i uniform integers in
  [lo, hi] (inclusive), int32.
* ``random_f32_dense``   fully connected, J_ij ~ N(0,1)*j_scale and
  h_i ~ N(0,1)*h_scale, drawn in float64 and cast to float32; the cast values
  are the instance.
* ``chimera_pm1``        Chimera-like sparse graph of rows x cols unit cells,
  each a K_{4,4} bipartite block, couplers uniform in {-1,+1}, h = 0, int32.
* ``batched_f32_dense``  a batch of dense float32 instances of uneven size,
  zero padded to N_max.
* ``logz_batch``         a batch of equal-size dense float32 instances.

Draw order (fixed, so that a seed names one instance): first the full N x N
coupling draw, of which the strict upper triangle is kept, then the length-N
field draw.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "random_int_dense", "random_f32_dense", "chimera_edges", "chimera_pm1",
    "batched_f32_dense", "logz_batch", "ferromagnet", "mattis",
    "free_spins_pow2_fields", "open_chain", "listing1_dict", "dict_to_dense",
    "workload",
]


def _upper(a: np.ndarray) -> np.ndarray:
    return np.triu(a, k=1)


def random_int_dense(N: int, seed: int, lo: int = -7, hi: int = 7):
    """Fully connected integer instance, values uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    J = _upper(rng.integers(lo, hi + 1, size=(N, N))).astype(np.int32)
    h = rng.integers(lo, hi + 1, size=N).astype(np.int32)
    return np.ascontiguousarray(J), np.ascontiguousarray(h)


def random_f32_dense(N: int, seed: int, j_scale: float | None = None,
                     h_scale: float = 0.1):
    """Fully connected float32 instance.

    ``j_scale`` defaults to 1/sqrt(N) (the N=48 dense workload); pass 1.0 for
    unscaled couplings.
    """
    if j_scale is None:
        j_scale = 1.0 / np.sqrt(N)
    rng = np.random.default_rng(seed)
    J = _upper(rng.standard_normal(size=(N, N)) * j_scale).astype(np.float32)
    h = (rng.standard_normal(size=N) * h_scale).astype(np.float32)
    return np.ascontiguousarray(J), np.ascontiguousarray(h)


def chimera_edges(rows: int, cols: int):
    """Edge list (i < j) of a rows x cols Chimera-like graph.

    Spin numbering v = 8*(cols*r + c) + 4*u + t with u in {0,1} (the two
    sides of the K_{4,4} cell) and t in 0..3.  Inside a cell every (u=0,t) is
    joined to every (u=1,t').  Side u=0 couples vertically to the same (t) in
    cell (r+1, c); side u=1 couples horizontally to the same (t) in cell
    (r, c+1).
    """
    def v(r, c, u, t):
        return 8 * (cols * r + c) + 4 * u + t

    edges = set()
    for r in range(rows):
        for c in range(cols):
            for t in range(4):
                for t2 in range(4):
                    edges.add(tuple(sorted((v(r, c, 0, t), v(r, c, 1, t2)))))
                if r + 1 < rows:
                    edges.add(tuple(sorted((v(r, c, 0, t), v(r + 1, c, 0, t)))))
                if c + 1 < cols:
                    edges.add(tuple(sorted((v(r, c, 1, t), v(r, c + 1, 1, t)))))
    return sorted(edges)


def chimera_pm1(rows: int, cols: int, seed: int):
    """Chimera-like instance with couplers uniform in {-1, +1}, h = 0."""
    N = 8 * rows * cols
    edges = chimera_edges(rows, cols)
    rng = np.random.default_rng(seed)
    vals = rng.choice(np.array([-1, 1]), size=len(edges))
    J = np.zeros((N, N), dtype=np.int32)
    for (i, j), val in zip(edges, vals):
        J[i, j] = val
    h = np.zeros(N, dtype=np.int32)
    return J, h


def batched_f32_dense(B: int, seed: int, n_lo: int = 16, n_hi: int = 32,
                      j_scale: float = 1.0, h_scale: float = 0.1):
    """B dense float32 instances with N_b uniform in [n_lo, n_hi].

    Returns (Ns int32[B], J float32[B, Nmax, Nmax], h float32[B, Nmax]) with
    zero padding beyond each N_b.
    """
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_lo, n_hi + 1, size=B).astype(np.int32)
    Nmax = int(n_hi)
    J = np.zeros((B, Nmax, Nmax), dtype=np.float32)
    h = np.zeros((B, Nmax), dtype=np.float32)
    for b in range(B):
        n = int(Ns[b])
        J[b, :n, :n] = _upper(rng.standard_normal(size=(n, n)) * j_scale)
        h[b, :n] = rng.standard_normal(size=n) * h_scale
    return Ns, J, h


def logz_batch(B: int, N: int, seed: int, j_scale: float | None = None,
               h_scale: float = 0.2):
    """B dense float32 instances of one size N (J ~ N(0,1)/sqrt(N) by default)."""
    if j_scale is None:
        j_scale = 1.0 / np.sqrt(N)
    rng = np.random.default_rng(seed)
    J = np.zeros((B, N, N), dtype=np.float32)
    h = np.zeros((B, N), dtype=np.float32)
    for b in range(B):
        J[b] = _upper(rng.standard_normal(size=(N, N)) * j_scale)
        h[b] = rng.standard_normal(size=N) * h_scale
    return J, h


def ferromagnet(N: int, Jval=1, dtype=np.int32):
    """Uniform coupling Jval on the complete graph, h = 0."""
    J = _upper(np.full((N, N), Jval)).astype(dtype)
    h = np.zeros(N, dtype=dtype)
    return J, h


def mattis(N: int, seed: int, Jval=1, dtype=np.int32):
    """Mattis instance J_ij = Jval * tau_i * tau_j, h = 0; returns (J, h, tau)."""
    rng = np.random.default_rng(seed)
    tau = rng.choice(np.array([-1, 1]), size=N)
    J = _upper(Jval * np.outer(tau, tau)).astype(dtype)
    h = np.zeros(N, dtype=dtype)
    return J, h, tau


def free_spins_pow2_fields(N: int, dtype=np.int32):
    """No couplings, h_i = 2^i."""
    J = np.zeros((N, N), dtype=dtype)
    h = (2 ** np.arange(N)).astype(dtype)
    return J, h


def open_chain(K, hvec=None, dtype=np.float64):
    """Open 1D chain: J_{i,i+1} = K[i]; optional fields."""
    K = np.asarray(K)
    N = len(K) + 1
    J = np.zeros((N, N), dtype=dtype)
    for i, k in enumerate(K):
        J[i, i + 1] = k
    h = np.zeros(N, dtype=dtype) if hvec is None else np.asarray(hvec, dtype=dtype)
    return J, h


def listing1_dict():
    """The two-spin graph dictionary of the paper's usage listing (1-based)."""
    return {(1, 1): -1.0, (1, 2): -0.2}


def dict_to_dense(graph: dict, N: int | None = None, dtype=np.float64):
    """Convert a 1-based {(i,j): value} graph to dense (J, h).

    Diagonal entries become fields h_i, off-diagonal entries couplings J_ij
    (stored at i<j); indices shift to 0-based.
    """
    if N is None:
        N = max(max(k) for k in graph)
    J = np.zeros((N, N), dtype=dtype)
    h = np.zeros(N, dtype=dtype)
    for (i, j), val in graph.items():
        i0, j0 = i - 1, j - 1
        if i0 == j0:
            h[i0] += val
        else:
            a, b = min(i0, j0), max(i0, j0)
            J[a, b] += val
    return J, h


def workload(name: str, seed: int | None = None):
    """The measured workloads, by name:
    "int24"       N=24 integer dense, S=100
    "dense48"     N=48 fp32 dense, S=1000
    "chimera48"   2x3-cell Chimera, J = +-1, h = 0, S=10000
    "batch4096"   4096 fp32 dense instances, N_b in [16, 32], S=64
    "logz256"     256 fp32 dense instances, N=28, beta in {0.5, 1, 2}, S=32"""
    if name == "int24":
        J, h = random_int_dense(24, 1 if seed is None else seed)
        return dict(N=24, J=J, h=h, S=100)
    if name == "dense48":
        J, h = random_f32_dense(48, 2 if seed is None else seed)
        return dict(N=48, J=J, h=h, S=1000)
    if name == "chimera48":
        J, h = chimera_pm1(2, 3, 3 if seed is None else seed)
        return dict(N=48, J=J, h=h, S=10000)
    if name == "batch4096":
        Ns, J, h = batched_f32_dense(4096, 4 if seed is None else seed)
        return dict(B=4096, Ns=Ns, J=J, h=h, S=64)
    if name == "logz256":
        J, h = logz_batch(256, 28, 5 if seed is None else seed)
        return dict(B=256, N=28, J=J, h=h, S=32,
                    beta=np.array([0.5, 1.0, 2.0], dtype=np.float32))
    raise ValueError(name)
