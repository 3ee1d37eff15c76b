"""Pins of the CPU oracle: checks against what the paper and the mathematics
fix, never against the oracle's own formula retyped.

Each ``pin_*`` takes the oracle module and raises AssertionError when the
oracle disagrees.  ``tests/test_oracle_pins.py`` runs them on the real oracle;
``tests/test_oracle_mutants.py`` runs them on copies of the oracle with
planted mistakes and requires that every mistake fails at least one pin.
"""

from __future__ import annotations

import math
import os
from itertools import combinations

import numpy as np

import instances as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(path):
    out = []
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                out.append(ln.split())
    return out


def _all_states_sorted(N, energy_of_mask):
    """All 2^N (E, mask) pairs sorted lexicographically (full sort)."""
    masks = np.arange(1 << N, dtype=np.int64)
    es = np.array([energy_of_mask(int(m)) for m in masks])
    order = np.lexsort((masks, es))
    return masks[order].astype(np.uint64), es[order]


def _popcount(x):
    return bin(int(x)).count("1")


# --------------------------------------------------------------- golden rows

def pin_listing1(orc):
    """Usage listing of Sec. 4.1, hand-derived from Eq. (1) (tests/golden)."""
    rows = _rows(os.path.join(GOLDEN, "listing1_n2.txt"))
    want_m = [int(r[0]) for r in rows]
    want_e = [float(r[1]) for r in rows]
    J, h = I.dict_to_dense(I.listing1_dict())
    m, e = orc.low_spectrum(J, h, 4)
    assert list(map(int, m)) == want_m, (m, want_m)
    assert np.allclose(e, want_e, atol=1e-12, rtol=0), (e, want_e)


def pin_encoding_eq5(orc):
    """Eq. (5) state #13 for N = 8: one-hot fields read each spin back."""
    rows = {r[0]: r[1:] for r in _rows(os.path.join(GOLDEN, "encoding_eq5.txt"))}
    N = int(rows["N"][0])
    mask = int(rows["mask"][0])
    spins = [int(s) for s in rows["spins"]]
    for i in range(N):
        J = np.zeros((N, N)); h = np.zeros(N); h[i] = 1.0
        # E = -h_i s_i = -s_i
        assert orc.energy(J, h, mask) == -spins[i], (i, orc.energy(J, h, mask))


# ------------------------------------------------------ independent formulas

def pin_qubo_identity(orc):
    """Eqs. (2)-(3): H(s) = F(q) + sum h - sum J for every state, with junk in
    the diagonal and lower triangle of J that both forms must ignore."""
    rng = np.random.default_rng(11)
    N = 9
    J, h = I.random_f32_dense(N, 7, j_scale=1.0, h_scale=0.7)
    J = J.astype(np.float64)
    J += np.tril(rng.standard_normal((N, N)) * 5.0)  # junk: diagonal + lower
    a, b, off = orc.qubo_from_ising(J, h)
    Ju = np.triu(J, 1)
    assert abs(off - (h.astype(np.float64).sum() - Ju.sum())) < 1e-12
    for m in range(1 << N):
        H = orc.energy(J, h, m)
        F = orc.qubo_energy(a, b, m)
        assert abs(H - (F + off)) < 1e-10, (m, H, F + off)


# ----------------------------------------------------------- brute force sort

def pin_full_sort(orc):
    """Heap selection equals the first S of a full sort of all 2^N states,
    with heavy ties (J in {-1,0,1}, h = 0) and with float couplings, for
    several thread counts and a sub-range."""
    N = 12
    rng = np.random.default_rng(5)
    Jt = np.triu(rng.integers(-1, 2, size=(N, N)), 1).astype(np.int32)
    ht = np.zeros(N, dtype=np.int32)
    Jf, hf = I.random_f32_dense(N, 9)
    for (J, h) in ((Jt, ht), (Jf, hf)):
        allm, alle = _all_states_sorted(N, lambda m: orc.energy(J, h, m))
        for S in (1, 37, 1 << N):
            for th in (1, 3):
                m, e = orc.low_spectrum(J, h, S, nthreads=th)
                assert len(m) == S
                assert np.array_equal(m, allm[:S]), (S, th)
                assert np.array_equal(e, alle[:S])
        lo, hi = 1000, 3001
        sub = (allm >= lo) & (allm < hi)
        m, e = orc.low_spectrum(J, h, 50, lo, hi, nthreads=4)
        assert np.array_equal(m, allm[sub][:50])


def pin_range_merge(orc):
    """Slices merge: top-S of [a,b) union top-S of [b,c) cut to S == top-S of [a,c)."""
    J, h = I.random_int_dense(14, 3)
    a, b, c, S = 100, 7000, 16384, 40
    m1, e1 = orc.low_spectrum(J, h, S, a, b)
    m2, e2 = orc.low_spectrum(J, h, S, b, c)
    mm = np.concatenate([m1, m2]); ee = np.concatenate([e1, e2])
    o = np.lexsort((mm, ee))[:S]
    m, e = orc.low_spectrum(J, h, S, a, c)
    assert np.array_equal(mm[o], m) and np.array_equal(ee[o], e)


# --------------------------------------------------------------- closed forms

def _ferro_energy(N, Jv, c):
    """Complete graph, uniform J, h = 0, c spins up: sum_{i<j} s_i s_j =
    (M^2 - N)/2 with M = 2c - N."""
    M = 2 * c - N
    return -Jv * (M * M - N) / 2


def pin_ferromagnet(orc):
    """Complete-graph ferromagnet: energy depends on the popcount only."""
    for N, Jv, dt in ((14, 1, np.int32), (13, 0.5, np.float64)):
        J, h = I.ferromagnet(N, Jv, dt)
        allm, alle = _all_states_sorted(N, lambda m: _ferro_energy(N, Jv, _popcount(m)))
        for S in (2, 2 + 2 * N, 500, 1 << N):
            m, e = orc.low_spectrum(J, h, S)
            assert np.array_equal(m, allm[:S]), (N, S)
            assert np.array_equal(np.asarray(e, dtype=np.float64), alle[:S].astype(np.float64))
        # ground level: exactly the two fully aligned states, E = -J N(N-1)/2
        m, e = orc.low_spectrum(J, h, 2)
        assert sorted(map(int, m)) == [0, (1 << N) - 1]
        assert e[0] == -Jv * N * (N - 1) / 2


def pin_mattis(orc):
    """Mattis J_ij = J tau_i tau_j: ferromagnet energies on m XOR tau-mask."""
    N = 13
    J, h, tau = I.mattis(N, 4)
    tmask = sum(1 << i for i in range(N) if tau[i] < 0)
    allm, alle = _all_states_sorted(N, lambda m: _ferro_energy(N, 1, _popcount(m ^ tmask)))
    m, e = orc.low_spectrum(J, h, 300)
    assert np.array_equal(m, allm[:300]) and np.array_equal(e, alle[:300].astype(np.int64))


def pin_free_pow2(orc):
    """J = 0, h_i = 2^i: the k-th lowest state is (2^N - 1) XOR k with energy
    -(2^N - 1) + 2k (no ties, so the order is fixed by the fields alone)."""
    N = 12
    J, h = I.free_spins_pow2_fields(N)
    m, e = orc.low_spectrum(J, h, 1 << N)
    k = np.arange(1 << N)
    assert np.array_equal(m.astype(np.int64), ((1 << N) - 1) ^ k)
    assert np.array_equal(e, -((1 << N) - 1) + 2 * k)


# ----------------------------------------------------------------- invariants

def pin_global_flip(orc):
    """h = 0: E(m) = E(~m); every level of the full spectrum has even size."""
    J, h = I.chimera_pm1(1, 2, 8)
    N = len(h)
    m, e = orc.low_spectrum(J, h, 1 << N)
    E = dict(zip(map(int, m), map(int, e)))
    full = (1 << N) - 1
    for mm, ee in E.items():
        assert E[full ^ mm] == ee
    _, counts = np.unique(e, return_counts=True)
    assert np.all(counts % 2 == 0)


def pin_gauge(orc):
    """Gauge transform J'_ij = t_i t_j J_ij, h'_i = t_i h_i maps state m to
    m XOR t-mask with the same energy, so the sorted energies agree exactly."""
    N = 10
    J, h = I.random_f32_dense(N, 12, j_scale=1.0, h_scale=0.5)
    t = np.random.default_rng(3).choice([-1.0, 1.0], size=N)
    J2 = np.triu(J.astype(np.float64) * np.outer(t, t), 1)
    h2 = h.astype(np.float64) * t
    tmask = sum(1 << i for i in range(N) if t[i] < 0)
    m1, e1 = orc.low_spectrum(J, h, 1 << N)
    m2, e2 = orc.low_spectrum(J2, h2, 1 << N)
    assert np.array_equal(e1, e2)
    mp = {int(a): float(b) for a, b in zip(m2, e2)}
    for a, b in zip(m1, e1):
        assert mp[int(a) ^ tmask] == b


# -------------------------------------------------------------------- log Z

def _chain_logz_transfer(K, hv, beta):
    """Open chain partition function by 2x2 transfer matrices (float64)."""
    s = np.array([-1.0, 1.0])
    v = np.exp(beta * hv[0] * s)
    for i, k in enumerate(K):
        T = np.exp(beta * k * np.outer(s, s))
        v = (v @ T) * np.exp(beta * hv[i + 1] * s)
    return math.log(v.sum())


def pin_chain_logz(orc):
    """Open chain: h = 0 closed form Z = 2 prod 2cosh(beta K_i), correlations
    <s_i s_j> = prod tanh(beta K_l); h != 0 against the transfer matrix."""
    rng = np.random.default_rng(21)
    K = rng.standard_normal(8)
    betas = np.array([0.3, 1.0, 1.7])
    J, h = I.open_chain(K)
    lz, e0, ms, mss = orc.logz(J, h, betas, moments=True)
    for b, beta in enumerate(betas):
        want = math.log(2.0) + sum(math.log(2 * math.cosh(beta * k)) for k in K)
        assert abs(lz[b] - want) < 1e-11 * max(1, abs(want)), (lz[b], want)
        assert np.allclose(ms[b], 0.0, atol=1e-12)
        for i, j in combinations(range(len(K) + 1), 2):
            want_c = np.prod(np.tanh(beta * K[i:j]))
            assert abs(mss[b, i, j] - want_c) < 1e-11, (i, j)
    hv = rng.standard_normal(len(K) + 1) * 0.6
    J, h = I.open_chain(K, hv)
    lz, _ = orc.logz(J, h, betas)
    for b, beta in enumerate(betas):
        want = _chain_logz_transfer(K, hv, beta)
        assert abs(lz[b] - want) < 1e-11 * max(1, abs(want))


def pin_free_logz(orc):
    """J = 0: log Z = sum log(2cosh(beta h_i)), <s_i> = tanh(beta h_i),
    <s_i s_j> = tanh(beta h_i) tanh(beta h_j)."""
    N = 9
    h = np.random.default_rng(2).standard_normal(N)
    J = np.zeros((N, N))
    betas = np.array([0.5, 2.0])
    lz, e0, ms, mss = orc.logz(J, h, betas, moments=True)
    assert abs(e0 - (-np.abs(h).sum())) < 1e-12
    for b, beta in enumerate(betas):
        assert abs(lz[b] - np.log(2 * np.cosh(beta * h)).sum()) < 1e-11
        t = np.tanh(beta * h)
        assert np.allclose(ms[b], t, atol=1e-12)
        assert np.allclose(np.triu(mss[b], 1), np.triu(np.outer(t, t), 1), atol=1e-12)


def pin_ferro_logz(orc):
    """Complete-graph ferromagnet: Z = sum_c C(N,c) exp(-beta E(c)) and
    <s_i s_j> = (<M^2> - N) / (N (N-1)) for every pair."""
    N, Jv = 12, 0.7
    J, h = I.ferromagnet(N, Jv, np.float64)
    betas = np.array([0.2, 1.0])
    lz, e0, ms, mss = orc.logz(J, h, betas, moments=True)
    for b, beta in enumerate(betas):
        w = np.array([math.comb(N, c) * math.exp(-beta * _ferro_energy(N, Jv, c))
                      for c in range(N + 1)])
        assert abs(lz[b] - math.log(w.sum())) < 1e-11 * abs(math.log(w.sum()))
        M2 = sum(w[c] * (2 * c - N) ** 2 for c in range(N + 1)) / w.sum()
        want = (M2 - N) / (N * (N - 1))
        assert np.allclose(mss[b][np.triu_indices(N, 1)], want, atol=1e-11)
        assert np.allclose(ms[b], 0.0, atol=1e-12)


def pin_logz_fd(orc):
    """Gradients of sum_b g_b log Z(beta_b) against central finite differences
    of the oracle's own log Z (a different code path: no moments involved)."""
    N = 7
    J, h = I.random_f32_dense(N, 31, j_scale=0.8, h_scale=0.4)
    J = J.astype(np.float64); h = h.astype(np.float64)
    betas = np.array([0.5, 1.0, 2.0]); g = np.array([0.3, -1.1, 0.7])
    gJ, gh = orc.logz_grad(J, h, betas, g)

    def f(Jx, hx):
        return float(np.dot(g, orc.logz(Jx, hx, betas)[0]))

    eps = 1e-5
    for i in range(N):
        hp = h.copy(); hp[i] += eps
        hm = h.copy(); hm[i] -= eps
        fd = (f(J, hp) - f(J, hm)) / (2 * eps)
        assert abs(fd - gh[i]) < 1e-7, (i, fd, gh[i])
    for i, j in combinations(range(N), 2):
        Jp = J.copy(); Jp[i, j] += eps
        Jm = J.copy(); Jm[i, j] -= eps
        fd = (f(Jp, h) - f(Jm, h)) / (2 * eps)
        assert abs(fd - gJ[i, j]) < 1e-7, (i, j, fd, gJ[i, j])
    assert np.all(np.tril(gJ) == 0.0)


def pin_logz_e0(orc):
    """The ground energy of the log Z pass equals the lowest energy of the
    search, and log Z(beta) -> -beta e0 + log(ground degeneracy) at large beta."""
    J, h = I.ferromagnet(10, 1.0, np.float64)
    lz, e0 = orc.logz(J, h, [40.0])
    m, e = orc.low_spectrum(J, h, 1)
    assert e0 == e[0]
    assert abs(lz[0] - (-40.0 * e0 + math.log(2.0))) < 1e-9


def pin_dos_ferromagnet(orc):
    """Density of states of the complete-graph ferromagnet: the C(N, c) states
    of popcount c share the energy -J((N - 2c)^2 - N)/2."""
    N = 12
    J, h = I.ferromagnet(N, 1, np.int32)
    e_min, counts = orc.density_of_states(J, h)
    want = np.zeros_like(counts)
    for c in range(N + 1):
        want[-((N - 2 * c) ** 2 - N) // 2 - e_min] += math.comb(N, c)
    assert np.array_equal(counts, want)
    assert int(counts.sum()) == 1 << N


def pin_dos_distinct_levels(orc):
    """Two instances whose 2^N energies are all distinct and known: free spins
    with h_i = 2^i (E = -(2^N - 1) + 2k, once each) and an open chain with
    |K_i| = 2^i, h = 0 (the 2^(N-1) bond patterns, each level twice)."""
    N = 10
    J, h = I.free_spins_pow2_fields(N)
    e_min, counts = orc.density_of_states(J, h)
    want = np.zeros_like(counts)
    for k in range(1 << N):
        want[-((1 << N) - 1) + 2 * k - e_min] += 1
    assert np.array_equal(counts, want)
    J = np.zeros((N, N), dtype=np.int32)
    for i in range(N - 1):
        J[i, i + 1] = (1 << i) * (1 if i % 3 else -1)
    h = np.zeros(N, dtype=np.int32)
    e_min, counts = orc.density_of_states(J, h)
    want = np.zeros_like(counts)
    for b in range(1 << (N - 1)):
        want[-((1 << (N - 1)) - 1) + 2 * b - e_min] += 2
    assert np.array_equal(counts, want)
    # a slice of the masks counts exactly that slice, whatever the thread split
    for nt in (0, 3):
        _, part = orc.density_of_states(J, h, e_min, len(counts), 256, 771, nthreads=nt)
        assert int(part.sum()) == 515
        assert np.all(part <= counts)


ALL_PINS = [
    pin_listing1, pin_encoding_eq5, pin_qubo_identity, pin_full_sort,
    pin_range_merge, pin_ferromagnet, pin_mattis, pin_free_pow2,
    pin_global_flip, pin_gauge, pin_chain_logz, pin_free_logz,
    pin_ferro_logz, pin_logz_fd, pin_logz_e0, pin_dos_ferromagnet, pin_dos_distinct_levels,
]
