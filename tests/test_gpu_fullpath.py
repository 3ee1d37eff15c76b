"""Oracle parity of the code paths the large workloads run, at oracle sizes.

The work plans give each lane only as many free spins as the device's lane
count leaves: an N = 24 search on the full device walks one 256-state block
per lane, and a log Z batch of a few instances has no high spins.  The test
hooks sg_debug_set_fill and sg_debug_set_batch_shift shrink the lane count the
plans assume, so these instances run the decompositions of the N = 48 search
(22 free spins per lane: the paired walk, block boundaries, high-spin fields,
fp32 re-anchors every 2^14 flips), of the upper batch levels (16 free spins)
and of the 256 x N = 28 log Z batch (14 free spins: records of 8 low spins
with 6 high spins in both walks; the gradient walk's sub-blocks of 6 give its
pair slots 8 high spins).  Every result is compared with the oracle state by
state: integer instances bit-exact, fp32 ones under the tolerance rules, log Z
within 1e-6 relative and gradients within 1e-5 of the largest entry, per
instance and inverse temperature.

The drift guard is checked on the same walks: the largest drift measured at a
re-anchor is positive and within the pruning margin, and a margin scaled below
the measured drift is reported as SG_EDRIFT without disturbing the next call.
"""

import contextlib

import numpy as np
import pytest

import instances as I
from parity import check_f32, check_int

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


@contextlib.contextmanager
def plan_fill(lanes):
    """Plans of the current stream assume `lanes` resident lanes."""
    from paper_1904_03621_amd import _lib
    _lib.check(_lib.sg_debug_set_fill(lanes), "sg_debug_set_fill")
    try:
        yield
    finally:
        _lib.check(_lib.sg_debug_set_fill(0), "sg_debug_set_fill")


@contextlib.contextmanager
def batch_shift(B, Nmax, S, shift):
    from paper_1904_03621_amd import _lib
    _lib.check(_lib.sg_debug_set_batch_shift(B, Nmax, S, shift), "sg_debug_set_batch_shift")
    try:
        yield
    finally:
        _lib.check(_lib.sg_debug_set_batch_shift(B, Nmax, S, -1), "sg_debug_set_batch_shift")


def to_dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def search(torch, J, h, S):
    import paper_1904_03621_amd as sg
    m, e = sg.low_spectrum(*to_dev(torch, J, h), S)
    info = sg.run_info()
    return m.cpu().numpy().astype(np.uint64), e.cpu().numpy(), info


def planned_free_bits(N, S, lanes):
    from paper_1904_03621_amd import _lib
    return max(n for _, n, _ in _lib.sg_debug_plan(N, S, 0, 1 << N, lanes))


def bound(J, h):
    return float(np.abs(np.triu(J.astype(np.float64), 1)).sum() + np.abs(h.astype(np.float64)).sum())


# ---------------------------------------------------------------- search

@pytest.mark.parametrize("N,S", [(20, 1000), (22, 1000), (24, 1000), (24, 50)])
def test_search_f32_full_walk(orc, torch_dev, N, S):
    """fp32 dense instances (the N = 48 workload's distribution) walked with
    up to 22 free spins per lane: margin > 0, the paired walk re-anchoring
    every 64 blocks."""
    J, h = I.random_f32_dense(N, 300 + N + S)
    with plan_fill(2):
        m, e, info = search(torch_dev, J, h, S)
    want_n = planned_free_bits(N, S, 2)
    assert info["free_bits_max"] == want_n >= N - 2, info
    om, oe = orc.low_spectrum(J, h, S)
    check_f32(N, J, m, e, om, oe, lambda x: orc.energy(J, h, x), "f32 N=%d fill 2" % N)
    # drift guard: the walk re-anchored (drift measured) inside its margin
    assert info["margin"] > 0.0
    assert 0.0 < info["max_drift"] <= info["margin"], info


@pytest.mark.parametrize("N,S,lanes,nmax", [(20, 100, 16, 15), (18, 100, 4, 15), (18, 600, 16, 13),
                                            (18, 20000, 4, 15), (16, 2000, 16, 11)])
@pytest.mark.parametrize("isint", [False, True])
def test_paired_walk_small_geometries(orc, torch_dev, N, S, lanes, nmax, isint):
    """The paired walks' smallest tables.  The chunks of a search double in
    size, so one search runs the plain walk (n = 8, 9 free spins), the paired
    walk over blocks of 8 (n = 10, 11: two and four block pairs per lane) and
    the one over blocks of 10 (n = 12 .. 15: two to sixteen pairs), in chunks
    that run with no threshold yet (every block re-walked; S = 20000 keeps the
    record open into the first chunk of blocks of 10) and in chunks with one
    (the fixed-point test decides)."""
    from paper_1904_03621_amd import _lib
    plan = _lib.sg_debug_plan(N, S, 0, 1 << N, lanes)
    assert max(n for _, n, _ in plan) == nmax, plan
    if isint:
        J, h = I.random_int_dense(N, 600 + N + lanes)
    else:
        J, h = I.random_f32_dense(N, 600 + N + lanes)
    with plan_fill(lanes):
        m, e, info = search(torch_dev, J, h, S)
    assert info["free_bits_max"] == nmax, info
    om, oe = orc.low_spectrum(J, h, S)
    if isint:
        check_int(m, e, om, oe, "paired N=%d lanes %d" % (N, lanes))
    else:
        check_f32(N, J, m, e, om, oe, lambda x: orc.energy(J, h, x),
                  "paired N=%d lanes %d" % (N, lanes))


@pytest.mark.parametrize("N,S,lanes,nmax", [(20, 100, 32, 14), (20, 5000, 8, 16),
                                            (22, 2000, 32, 16), (21, 100, 8, 17),
                                            (22, 300, 8, 18), (22, 100, 4, 19)])
@pytest.mark.parametrize("isint", [False, True])
def test_three_field_walk(orc, torch_dev, N, S, lanes, nmax, isint):
    """The three-field walk (chunks with n >= 14 free spins walk three blocks
    of 10 per word): one level of triples and a tail of four blocks (n = 14),
    two levels and a tail of two (n = 15, 17), two and three levels with
    tails of four (n = 16, 18), four levels and a tail of two (n = 19), with
    and without a threshold yet (S = 5000 keeps the record open into the
    first chunks of n >= 14)."""
    from paper_1904_03621_amd import _lib
    plan = _lib.sg_debug_plan(N, S, 0, 1 << N, lanes)
    assert max(n for _, n, _ in plan) == nmax, plan
    if isint:
        J, h = I.random_int_dense(N, 700 + N + lanes)
    else:
        J, h = I.random_f32_dense(N, 700 + N + lanes)
    with plan_fill(lanes):
        m, e, info = search(torch_dev, J, h, S)
    assert info["free_bits_max"] == nmax, info
    om, oe = orc.low_spectrum(J, h, S)
    if isint:
        check_int(m, e, om, oe, "three-field N=%d lanes %d" % (N, lanes))
    else:
        check_f32(N, J, m, e, om, oe, lambda x: orc.energy(J, h, x),
                  "three-field N=%d lanes %d" % (N, lanes))


@pytest.mark.parametrize("N,S,seed", [(22, 100, 1), (24, 100, 2), (24, 1000, 3)])
def test_search_int32_walk_full(orc, torch_dev, N, S, seed):
    """Integer couplings of up to 2^20: the walk runs in int32 (its values
    exceed fp32's 24 bits), here with up to 22 free spins per lane."""
    J, h = I.random_int_dense(N, 400 + seed, lo=-(1 << 20), hi=1 << 20)
    Bv = bound(J, h)
    assert 2.1 * Bv >= 2.0 ** 24 and Bv < 2.0 ** 28, "instance not on the int32 walk"
    with plan_fill(2):
        m, e, info = search(torch_dev, J, h, S)
    assert info["free_bits_max"] == planned_free_bits(N, S, 2) >= N - 2, info
    om, oe = orc.low_spectrum(J, h, S)
    check_int(m, e, om, oe, "int32 walk N=%d" % N)


@pytest.mark.parametrize("lanes", [2, 64, 4096])
def test_int24_workload_full_walk(orc, torch_dev, lanes):
    """The N = 24 integer workload (exact fp32 walk) at three decompositions."""
    w = I.workload("int24")
    with plan_fill(lanes):
        m, e, info = search(torch_dev, w["J"], w["h"], w["S"])
    assert info["free_bits_max"] == planned_free_bits(24, w["S"], lanes)
    om, oe = orc.low_spectrum(w["J"], w["h"], w["S"])
    check_int(m, e, om, oe, "int24 fill %d" % lanes)


def test_chimera24_full_walk(orc, torch_dev):
    """A 1 x 3-cell Chimera instance (24 spins, J = +-1, h = 0) with S = 10000,
    the sparse workload's structure and S, walked with 22 free spins."""
    J, h = I.chimera_pm1(1, 3, 5)
    S = 10000
    with plan_fill(2):
        m, e, info = search(torch_dev, J, h, S)
    assert info["free_bits_max"] == 22
    om, oe = orc.low_spectrum(J, h, S)
    check_int(m, e, om, oe, "chimera 1x3 fill 2")


def test_range_slice_full_walk(orc, torch_dev):
    """A mask range of an N = 40 instance walked with 22 free spins per lane
    (the slice a multi-device run would give one device)."""
    N, S = 40, 300
    J, h = I.random_f32_dense(N, 77)
    lo, hi = 5 << 22, 7 << 22
    import paper_1904_03621_amd as sg
    with plan_fill(1):
        m, e = sg.low_spectrum_range(*to_dev(torch_dev, J, h), S, lo, hi)
        info = sg.run_info()
    assert info["free_bits_max"] == 22
    m, e = m.cpu().numpy().astype(np.uint64), e.cpu().numpy()
    om, oe = orc.low_spectrum(J, h, S, lo, hi)
    check_f32(N, J, m, e, om, oe, lambda x: orc.energy(J, h, x), "N=40 slice")
    assert 0.0 < info["max_drift"] <= info["margin"]


# ------------------------------------------------------------ drift guard

def test_drift_guard_reports_and_clears(orc, torch_dev):
    """A margin scaled below the measured drift raises SG_EDRIFT; the next
    call on the stream (margin restored) is clean and correct."""
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    N, S = 24, 200
    J, h = I.random_f32_dense(N, 91)
    Jt, ht = to_dev(torch_dev, J, h)
    with plan_fill(2):
        sg.low_spectrum(Jt, ht, S)
        info = sg.run_info()
        drift, margin = info["max_drift"], info["margin"]
        assert 0.0 < drift <= margin
        scale = 0.25 * drift / margin
        _lib.check(_lib.sg_debug_set_margin_scale(scale), "sg_debug_set_margin_scale")
        try:
            sg.low_spectrum(Jt, ht, S, check=False)
            st = _lib.sg_get_error()
            info2 = sg.run_info()
        finally:
            _lib.check(_lib.sg_debug_set_margin_scale(1.0), "sg_debug_set_margin_scale")
        assert st == _lib.SG_EDRIFT, _lib.STATUS_NAMES.get(st, st)
        assert info2["margin"] < info2["max_drift"]
        # the error was read and cleared; the next call is clean
        m, e = sg.low_spectrum(Jt, ht, S, check=False)
        assert _lib.sg_get_error() == _lib.SG_OK
    om, oe = orc.low_spectrum(J, h, S)
    check_f32(N, J, m.cpu().numpy().astype(np.uint64), e.cpu().numpy(), om, oe,
              lambda x: orc.energy(J, h, x), "after drift error")


# --------------------------------------------------------------- batched

@pytest.mark.parametrize("isint", [True, False])
def test_batched_upper_levels(orc, torch_dev, isint):
    """A small batch with the level geometry of the 4096-instance workload's
    upper levels: lanes of 16 free spins (blocks of 256 states, re-anchors),
    each instance against the oracle and against the single search."""
    import paper_1904_03621_amd as sg
    B, S, Nmax = 6, 64, 22
    rng = np.random.default_rng(55 + isint)
    Ns = np.array([22, 16, 21, 19, 22, 17], dtype=np.int32)
    dt = np.int32 if isint else np.float32
    J = np.zeros((B, Nmax, Nmax), dtype=dt)
    h = np.zeros((B, Nmax), dtype=dt)
    for b in range(B):
        n = int(Ns[b])
        seed = int(rng.integers(1 << 30))
        if isint:
            Jb, hb = I.random_int_dense(n, seed)
        else:
            Jb, hb = I.random_f32_dense(n, seed, j_scale=1.0, h_scale=0.1)
        J[b, :n, :n], h[b, :n] = Jb, hb
    with batch_shift(B, Nmax, S, 5):
        bm, be = sg.low_spectrum_batched(*to_dev(torch_dev, Ns, J, h), S)
        info = sg.run_info()
    assert info["free_bits_max"] == 16, info
    bm, be = bm.cpu().numpy().astype(np.uint64), be.cpu().numpy()
    for b in range(B):
        n = int(Ns[b])
        Jb, hb = J[b, :n, :n], h[b, :n]
        om, oe = orc.low_spectrum(Jb, hb, S)
        if isint:
            check_int(bm[b], be[b], om, oe, "batch b=%d" % b)
        else:
            check_f32(n, Jb, bm[b], be[b], om, oe, lambda x: orc.energy(Jb, hb, x),
                      "batch b=%d" % b)
        sm, se, _ = search(torch_dev, Jb, hb, S)
        assert np.array_equal(sm, bm[b]) and np.array_equal(se, be[b]), "b=%d" % b


# ------------------------------------------------------------------ log Z

BETAS = np.array([0.5, 1.0, 2.0], dtype=np.float32)


def gpu_logz_per_beta(torch, J, h, betas):
    """log Z [B, K] and, for every beta k, the gradient of log Z(beta_k):
    grad_J [K, B, N, N], grad_h [K, B, N]."""
    import paper_1904_03621_amd as sg
    Jt, ht, bt = to_dev(torch, J, h, betas)
    lz, e0, _, _ = sg.logz_forward(Jt, ht, bt, 8)
    B, K = lz.shape
    gJ, gh = [], []
    for k in range(K):
        g = torch.zeros((B, K), dtype=torch.float64, device=lz.device)
        g[:, k] = 1.0
        a, c = sg.logz_backward(Jt, ht, bt, e0, lz, g)
        gJ.append(a.cpu().numpy().astype(np.float64))
        gh.append(c.cpu().numpy().astype(np.float64))
    return lz.cpu().numpy(), np.stack(gJ), np.stack(gh)


def check_against_moments(lz, gJ, gh, J, h, betas, orc, what):
    """R13 per inverse temperature: |d log Z| <= 1e-6 |log Z|; every gradient
    entry within 1e-5 of the largest oracle entry, grad_J zero on and below
    the diagonal."""
    N = len(h)
    lz_ref, _, ms, mss = orc.logz(J, h, betas, moments=True)
    iu = np.triu_indices(N, 1)
    low = np.tril_indices(N)
    for k, bk in enumerate(betas):
        assert abs(lz[k] - lz_ref[k]) <= 1e-6 * abs(lz_ref[k]), (what, k, lz[k], lz_ref[k])
        rJ = float(bk) * mss[k]
        rh = float(bk) * ms[k]
        scale = max(np.abs(rJ[iu]).max(), np.abs(rh).max())
        eJ = np.abs(gJ[k][iu] - rJ[iu]).max() / scale
        eh = np.abs(gh[k] - rh).max() / scale
        assert eJ <= 1e-5 and eh <= 1e-5, "%s beta=%g: grad err J %.3g h %.3g" % (what, bk, eJ, eh)
        assert np.all(gJ[k][low] == 0.0)


@pytest.mark.parametrize("N", [16, 20])
def test_logz_high_spin_walk(orc, torch_dev, N):
    """14 free spins per lane (as at the 256 x N = 28 workload): the partition
    sums take records of 10 low spins with 4 high spins, two blocks at a time;
    the gradient walk takes records of 8 with 6 high spins, and its sub-blocks
    of 6 give its low-high and high-high pair slots 8 high spins."""
    B = 2
    J, h = I.logz_batch(B, N, 500 + N)
    with plan_fill(1):
        lz, gJ, gh = gpu_logz_per_beta(torch_dev, J, h, BETAS)
    for b in range(B):
        check_against_moments(lz[b], gJ[:, b], gh[:, b], J[b], h[b], BETAS, orc,
                              "N=%d b=%d" % (N, b))


@pytest.mark.parametrize("N,betas", [(11, [1.0]), (12, [0.5, 2.0]), (13, [0.5, 1.0, 2.0]),
                                     (18, [0.7]), (22, [0.5, 1.5])])
def test_logz_paired_blocks(orc, torch_dev, N, betas):
    """The partition sums over records of 10 walk a lane's blocks in pairs:
    2, 4, 8 and 16 blocks per lane (N = 11, 12, 13 and N >= 14 with every
    spin from 10 up free), for one, two and three beta, against the oracle's
    log Z (1e-6 relative)."""
    import paper_1904_03621_amd as sg
    B = 2
    J, h = I.logz_batch(B, N, 700 + N)
    bt = np.asarray(betas, dtype=np.float32)
    Jt, ht, btt = to_dev(torch_dev, J, h, bt)
    with plan_fill(1):
        lz, _, _, _ = sg.logz_forward(Jt, ht, btt, 4)
    lz = lz.cpu().numpy()
    for b in range(B):
        ref, _ = orc.logz(J[b], h[b], bt)
        for k in range(len(bt)):
            assert abs(lz[b, k] - ref[k]) <= 1e-6 * abs(ref[k]), (N, b, k, lz[b, k], ref[k])


@pytest.mark.timeout(900)
def test_logz_workload_instance0(orc, torch_dev):
    """The 256 x N = 28 workload as run by the benchmark (14 free spins per
    lane; the partition sums over pairs of records of 10, the gradient walk
    over records of 8): instance 0's log Z and both gradients at each beta
    against the oracle, entry by entry."""
    w = I.workload("logz256")
    lz, gJ, gh = gpu_logz_per_beta(torch_dev, w["J"], w["h"], w["beta"])
    check_against_moments(lz[0], gJ[:, 0], gh[:, 0], w["J"][0], w["h"][0], w["beta"], orc,
                          "logz256 b=0")
