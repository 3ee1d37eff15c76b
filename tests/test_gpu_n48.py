"""Full-size (N = 48, all 2^48 states) GPU searches, checked where the oracle
cannot enumerate the whole space:

* closed forms whose lowest states are spread over the entire mask space
  (complete-graph ferromagnet in int32 and fp32, Mattis gauge of it, uniform
  field), compared element by element;
* the dense fp32 benchmark workload: every returned energy against the
  oracle, and oracle slices of 2^22 states around returned states, both
  against the full result and against the range search of the same slice;
* the Chimera +-1 workload (S = 10000): exact energies, exact slices, the
  global-flip pairing of every complete level, gauge invariance, and every
  complete level's size against the exact density of states of the instance;
* invariances of the dense fp32 workload: a gauge transform (bit-identical
  energies), a spin permutation (energies within the tolerance) and the
  prefix property in S (the 100 lowest are the first 100 of the 1000 lowest);
* the drift guard on the benchmark search (measured drift within the margin).
"""

import itertools

import numpy as np
import pytest

import instances as I
from parity import check_f32, check_int, sorted_by_key, tau_of

pytestmark = pytest.mark.gpu

N = 48
FULL = (1 << N) - 1


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def gpu_search(torch, J, h, S, lo=None, hi=None, info=False):
    import paper_1904_03621_amd as sg
    Jt = torch.from_numpy(np.ascontiguousarray(J)).cuda()
    ht = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    if lo is None:
        m, e = sg.low_spectrum(Jt, ht, S)
    else:
        m, e = sg.low_spectrum_range(Jt, ht, S, lo, hi)
    out = (m.cpu().numpy().astype(np.uint64), e.cpu().numpy())
    return out + (sg.run_info(),) if info else out


@pytest.fixture(scope="module")
def dense48(torch_dev):
    """The benchmark instance (N = 48 dense fp32, seed 2, S = 1000), searched once."""
    J, h = I.random_f32_dense(N, 2)
    m, e, info = gpu_search(torch_dev, J, h, 1000, info=True)
    return J, h, m, e, info


@pytest.fixture(scope="module")
def chimera48(torch_dev):
    """Chimera 2x3 cells (48 spins), couplers +-1, h = 0, S = 10000, searched once."""
    J, h = I.chimera_pm1(2, 3, 3)
    m, e = gpu_search(torch_dev, J, h, 10000)
    return J, h, m, e.astype(np.int64)


def popcount_masks(N, c):
    out = []
    for bits in itertools.combinations(range(N), c):
        out.append(sum(1 << b for b in bits))
    return out


def ferro_expected(N, S, Jv, xor=0):
    """Lowest S of the complete-graph ferromagnet (optionally gauge-shifted by
    xor): levels by |2c - N| descending, masks ascending inside a level."""
    rows = []
    r = 0
    while len(rows) < S:
        lvl = set(popcount_masks(N, r)) | set(FULL ^ m for m in popcount_masks(N, r))
        M = N - 2 * r
        E = -Jv * (M * M - N) / 2
        rows += sorted((E, m ^ xor) for m in lvl)
        r += 1
    rows.sort()
    rows = rows[:S]
    return np.array([m for _, m in rows], dtype=np.uint64), np.array([e for e, _ in rows])


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_ferromagnet_closed_form(torch_dev, dtype):
    J, h = I.ferromagnet(N, 1, dtype)
    S = 1000
    m, e = gpu_search(torch_dev, J, h, S)
    wm, we = ferro_expected(N, S, 1)
    assert np.array_equal(m, wm)
    assert np.array_equal(e.astype(np.float64), we)


def test_mattis_closed_form(torch_dev):
    J, h, tau = I.mattis(N, 9)
    tmask = sum(1 << i for i in range(N) if tau[i] < 0)
    S = 500
    m, e = gpu_search(torch_dev, J, h, S)
    # energies are those of the ferromagnet; the states are XORed by tmask,
    # which reorders masks inside each level
    rows = []
    for r in range(3):
        lvl = set(popcount_masks(N, r)) | set(FULL ^ x for x in popcount_masks(N, r))
        M = N - 2 * r
        rows += [(-(M * M - N) // 2, x ^ tmask) for x in lvl]
    rows.sort()
    wm = np.array([x for _, x in rows[:S]], dtype=np.uint64)
    we = np.array([x for x, _ in rows[:S]])
    assert np.array_equal(e.astype(np.int64), we)
    assert np.array_equal(m, wm)


def test_uniform_field_closed_form(torch_dev):
    """J = 0, h_i = 1: E = N - 2 popcount; levels of 1, 48, 1128 states."""
    J = np.zeros((N, N), dtype=np.int32)
    h = np.ones(N, dtype=np.int32)
    S = 1000
    m, e = gpu_search(torch_dev, J, h, S)
    want = [FULL] + sorted(FULL ^ (1 << b) for b in range(N))
    want += sorted(FULL ^ x for x in popcount_masks(N, 2))
    want = np.array(want[:S], dtype=np.uint64)
    assert np.array_equal(m, want)
    pc = np.array([bin(int(x)).count("1") for x in m])
    assert np.array_equal(e.astype(np.int64), N - 2 * pc)


def _slices_around(masks, picks, width_log=22):
    out = []
    for k in picks:
        lo = (int(masks[k]) >> width_log) << width_log
        out.append((lo, lo + (1 << width_log)))
    return out


def test_dense_f32_workload(orc, torch_dev, dense48):
    """The benchmark instance: N = 48 dense fp32, seed 2, S = 1000."""
    J, h, m, e, _ = dense48
    S = 1000
    tau = tau_of(J)
    assert len(set(m.tolist())) == S and int(m.max()) < (1 << N)
    assert sorted_by_key(m, e)
    eo = np.array([orc.energy(J, h, int(x)) for x in m])
    assert np.max(np.abs(eo - e)) <= tau
    T = float(e[-1])
    G = set(m.tolist())
    for (lo, hi) in _slices_around(m, [0, S // 2, S - 1]):
        om, oe = orc.low_spectrum(J, h, S, lo, hi)
        for x, ex in zip(om.tolist(), oe):
            if ex < T - 2 * tau:
                assert x in G, "slice state %d (E=%.7f) below T=%.7f missing" % (x, ex, T)
        rm, re_ = gpu_search(torch_dev, J, h, S, lo, hi)
        check_f32(N, J, rm, re_, om, oe, lambda x: orc.energy(J, h, x), "slice %d" % lo)


def test_chimera_workload(orc, torch_dev, chimera48):
    """Chimera 2x3 cells (48 spins), couplers +-1, h = 0, S = 10000."""
    J, h, m, e = chimera48
    S = 10000
    assert len(set(m.tolist())) == S and sorted_by_key(m, e)
    eo = np.array([orc.energy(J, h, int(x)) for x in m])
    assert np.array_equal(eo, e)
    # global flip: every level below the last one is closed under complement
    G = set(m.tolist())
    last = e[-1]
    for x, ex in zip(m.tolist(), e):
        if ex < last:
            assert (FULL ^ x) in G
    Tkey = (int(e[-1]), int(m[-1]))
    for (lo, hi) in _slices_around(m, [0, S // 3, S - 1]):
        om, oe = orc.low_spectrum(J, h, S, lo, hi)
        in_slice = sorted((int(ex), x) for x, ex in zip(m.tolist(), e) if lo <= x < hi)
        okeys = [(int(ex), int(x)) for x, ex in zip(om.tolist(), oe)]
        cut = min(Tkey, okeys[-1]) if len(okeys) == S else Tkey
        want = [k for k in okeys if k <= cut]
        got = [(ex, x) for ex, x in in_slice if (ex, x) <= cut]
        assert got == want, "slice %d differs" % lo
        rm, re_ = gpu_search(torch_dev, J, h, S, lo, hi)
        check_int(rm, re_, om, oe, "chimera slice %d" % lo)


def test_chimera_gauge_invariance(torch_dev):
    J, h = I.chimera_pm1(2, 3, 3)
    S = 2000
    m1, e1 = gpu_search(torch_dev, J, h, S)
    t = np.random.default_rng(17).choice([-1, 1], size=N)
    J2 = (J * np.outer(t, t)).astype(np.int32)
    m2, e2 = gpu_search(torch_dev, J2, h, S)
    assert np.array_equal(e1, e2)
    tmask = sum(1 << i for i in range(N) if t[i] < 0)
    # complete levels map onto each other state by state
    last = e1[-1]
    s1 = set(int(x) ^ tmask for x, ex in zip(m1, e1) if ex < last)
    s2 = set(int(x) for x, ex in zip(m2, e2) if ex < last)
    assert s1 == s2


def test_chimera_levels_vs_density_of_states(torch_dev, chimera48):
    """Exactness of the S = 10000 Chimera search against the exact density of
    states of the same instance (all 2^48 states counted): every complete
    level of the result holds exactly the level's count of states, the cut
    level no more; the counts sum to 2^48 and are all even (global flip)."""
    import paper_1904_03621_amd as sg
    J, h, m, e = chimera48
    Jt, ht = (torch_dev.from_numpy(np.ascontiguousarray(x)).cuda() for x in (J, h))
    e_min, counts = sg.density_of_states(Jt, ht)
    counts = counts.cpu().numpy().astype(np.uint64)
    assert int(counts.sum(dtype=np.uint64)) == 1 << N
    assert np.all(counts % 2 == 0)
    levels, sizes = np.unique(e, return_counts=True)
    assert levels[0] == e_min + int(np.nonzero(counts)[0][0]), "ground level differs"
    for lv, sz in zip(levels[:-1], sizes[:-1]):
        assert counts[lv - e_min] == sz, "level %d: %d states found, %d exist" % (
            lv, sz, counts[lv - e_min])
    assert counts[levels[-1] - e_min] >= sizes[-1]
    # no state between two returned levels was skipped
    nz = np.nonzero(counts)[0] + e_min
    assert np.array_equal(nz[:len(levels)], levels)


def _equal_energy_groups(m, e):
    """{energy: set of masks} of a sorted result, without its last (cut) group."""
    groups = {}
    for x, ex in zip(m.tolist(), e.tolist()):
        groups.setdefault(ex, set()).add(x)
    groups.pop(e.tolist()[-1])
    return groups


def test_dense48_gauge_invariance(torch_dev, dense48):
    """J' = t_i t_j J, h' = t_i h (t = +-1): the fp64 rescoring is exact under
    the sign change, so the energy lists are bit-identical and each energy
    group maps onto the other by XOR with the mask of t = -1."""
    J, h, m1, e1, _ = dense48
    t = np.random.default_rng(23).choice([-1, 1], size=N)
    J2 = (J * np.outer(t, t)).astype(np.float32)
    h2 = (h * t).astype(np.float32)
    m2, e2 = gpu_search(torch_dev, J2, h2, 1000)
    assert np.array_equal(e1.view(np.uint32), e2.view(np.uint32)), "energy bits differ"
    tmask = sum(1 << i for i in range(N) if t[i] < 0)
    g1 = _equal_energy_groups(m1, e1)
    g2 = _equal_energy_groups(m2, e2)
    assert g1.keys() == g2.keys()
    for ex in g1:
        assert {x ^ tmask for x in g1[ex]} == g2[ex]


def test_dense48_permutation_invariance(orc, torch_dev, dense48):
    """Spin i renamed pi(i): the same states (bits moved by pi) with the same
    energies up to the summation order (within the tolerance), the sets equal
    apart from states within 2 tau of the S-th energy."""
    J, h, m1, e1, _ = dense48
    pi = np.random.default_rng(29).permutation(N)
    Jf = np.triu(J.astype(np.float64), 1)
    Jf = Jf + Jf.T
    J2 = np.zeros((N, N), dtype=np.float64)
    h2 = np.zeros(N, dtype=np.float64)
    for i in range(N):
        h2[pi[i]] = h[i]
        for j in range(N):
            J2[pi[i], pi[j]] = Jf[i, j]
    J2 = np.triu(J2, 1).astype(np.float32)
    h2 = h2.astype(np.float32)
    m2, e2 = gpu_search(torch_dev, J2, h2, 1000)

    def moved(x):
        return sum(1 << int(pi[i]) for i in range(N) if (x >> i) & 1)

    tau = tau_of(J)
    mapped = {moved(x): ex for x, ex in zip(m1.tolist(), e1.tolist())}
    T = float(e1[-1])
    G2 = dict(zip(m2.tolist(), e2.tolist()))
    for x, ex in mapped.items():
        if x in G2:
            assert abs(G2[x] - ex) <= tau
        else:
            assert ex >= T - 2 * tau, "state %d at %.7f missing after the permutation" % (x, ex)
    for x, ex in G2.items():
        if x not in mapped:
            assert ex <= T + 2 * tau
            assert abs(orc.energy(J2, h2, x) - ex) <= tau


def test_dense48_s_prefix(torch_dev, dense48):
    """The search is exact, so its 100 lowest states are the first 100 of its
    1000 lowest, bit for bit."""
    J, h, m1, e1, _ = dense48
    m2, e2 = gpu_search(torch_dev, J, h, 100)
    assert np.array_equal(m2, m1[:100])
    assert np.array_equal(e2.view(np.uint32), e1[:100].view(np.uint32))


def test_dense48_drift_guard(dense48):
    """The benchmark search re-anchors every 2^10 flips: its largest measured
    drift is positive and within the pruning margin (no SG_EDRIFT)."""
    _, _, _, _, info = dense48
    assert info["free_bits_max"] == 22
    assert 0.0 < info["max_drift"] <= info["margin"], info
