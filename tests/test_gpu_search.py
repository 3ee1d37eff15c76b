"""GPU search against the CPU oracle at sizes the oracle finishes in seconds:
every state of tiny instances, the N = 24 integer workload bit-exact, heavy
ties, float instances under the tolerance rules, mask-range slices, closed
forms, error paths and determinism."""

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


def gpu_search(torch, J, h, S, lo=None, hi=None):
    import paper_1904_03621_amd as sg
    Jt = torch.from_numpy(np.ascontiguousarray(J)).cuda()
    ht = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    if lo is None:
        m, e = sg.low_spectrum(Jt, ht, S)
    else:
        m, e = sg.low_spectrum_range(Jt, ht, S, lo, hi)
    return m.cpu().numpy().astype(np.uint64), e.cpu().numpy()


def compare(orc, torch, J, h, S, lo=None, hi=None, what=""):
    N = len(h)
    m, e = gpu_search(torch, J, h, S, lo, hi)
    om, oe = orc.low_spectrum(J, h, S, 0 if lo is None else lo, None if hi is None else hi)
    if orc.is_integer_instance(J, h):
        check_int(m, e, om, oe, what)
    else:
        check_f32(N, J, m, e, om, oe, lambda x: orc.energy(J, h, x), what)
    return m, e


def test_listing1(orc, torch_dev):
    J, h = I.dict_to_dense(I.listing1_dict())
    m, e = gpu_search(torch_dev, J.astype(np.float32), h.astype(np.float32), 4)
    assert list(map(int, m)) == [2, 0, 1, 3]
    assert np.allclose(e, [-1.2, -0.8, 0.8, 1.2], atol=1e-6)


@pytest.mark.parametrize("N", list(range(1, 13)) + [15, 16, 17])
def test_every_state_int(orc, torch_dev, N):
    J, h = I.random_int_dense(N, 100 + N)
    compare(orc, torch_dev, J, h, 1 << N, what="int N=%d all" % N)


@pytest.mark.parametrize("N", [1, 3, 5, 6, 7, 9, 12, 14, 15, 16, 17])
def test_every_state_f32(orc, torch_dev, N):
    """Every state returned in order; N = 15 walks blocks of 7 low spins,
    N >= 16 blocks of 8."""
    J, h = I.random_f32_dense(N, 200 + N, j_scale=1.0, h_scale=0.3)
    compare(orc, torch_dev, J, h, 1 << N, what="f32 N=%d all" % N)


@pytest.mark.parametrize("seed", [1, 11, 12])
def test_n24_integer_bit_exact(orc, torch_dev, seed):
    """The N = 24 workload: J_ij, h_i uniform integers in [-7, 7], S = 100."""
    J, h = I.random_int_dense(24, seed)
    compare(orc, torch_dev, J, h, 100, what="N=24 seed %d" % seed)


def test_heavy_ties_int(orc, torch_dev):
    N = 22
    rng = np.random.default_rng(8)
    J = np.triu(rng.integers(-1, 2, size=(N, N)), 1).astype(np.int32)
    h = np.zeros(N, dtype=np.int32)
    compare(orc, torch_dev, J, h, 5000, what="ties N=22")


def test_chimera_small_int(orc, torch_dev):
    J, h = I.chimera_pm1(1, 3, 5)  # 24 spins
    m, e = compare(orc, torch_dev, J, h, 3000, what="chimera 1x3")
    full = (1 << 24) - 1
    ms = set(map(int, m))
    top = e[-1]
    for x, ex in zip(map(int, m), e):
        if ex < top:
            assert (full ^ x) in ms, "global flip partner missing"


@pytest.mark.parametrize("seed", [2, 21])
def test_dense_f32_n24(orc, torch_dev, seed):
    J, h = I.random_f32_dense(24, seed)
    compare(orc, torch_dev, J, h, 1000, what="f32 N=24 seed %d" % seed)


def test_unscaled_f32_n22(orc, torch_dev):
    J, h = I.random_f32_dense(22, 4, j_scale=1.0, h_scale=0.1)
    compare(orc, torch_dev, J, h, 64, what="f32 unscaled N=22")


def test_ferromagnet_f32_exact_ties(orc, torch_dev):
    """fp32 couplings with massive exact degeneracy (J = 1.0)."""
    J, h = I.ferromagnet(20, 1.0, np.float32)
    m, e = gpu_search(torch_dev, J, h, 300)
    om, oe = orc.low_spectrum(J, h, 300)
    assert np.array_equal(m, om) and np.array_equal(e.astype(np.float64), oe)


def test_exact_f32_degenerate(orc, torch_dev):
    """fp32 instances whose arithmetic is exact (all values on one dyadic
    grid) run with a zero margin and the integer tie rule: an all-zero
    instance returns the S smallest masks, a dyadic one matches the oracle
    bit for bit."""
    N = 30
    J = np.zeros((N, N), dtype=np.float32)
    h = np.zeros(N, dtype=np.float32)
    m, e = gpu_search(torch_dev, J, h, 100)
    assert np.array_equal(m, np.arange(100, dtype=np.uint64)) and np.all(e == 0)
    N = 22
    rng = np.random.default_rng(33)
    J = np.triu(rng.integers(-4, 5, size=(N, N)) * 0.25, 1).astype(np.float32)
    h = (rng.integers(-4, 5, size=N) * 0.125).astype(np.float32)
    m, e = gpu_search(torch_dev, J, h, 2000)
    om, oe = orc.low_spectrum(J, h, 2000)
    assert np.array_equal(m, om) and np.array_equal(e.astype(np.float64), oe)


@pytest.mark.parametrize("isint", [True, False])
def test_range_slices(orc, torch_dev, isint):
    N = 32
    if isint:
        J, h = I.random_int_dense(N, 77)
    else:
        J, h = I.random_f32_dense(N, 78)
    for lo in [0, (1 << 31) + (5 << 25), (1 << 32) - (1 << 23)]:
        hi = lo + (1 << 23)
        compare(orc, torch_dev, J, h, 200, lo, hi, what="N=32 slice %d" % lo)
    # a range whose ends are only 64-aligned
    lo = 64 * 1234567
    compare(orc, torch_dev, J, h, 50, lo, lo + 64 * 40000, what="N=32 ragged slice")


def test_pow2_fields_closed_form(torch_dev):
    """J = 0, h_i = 2^i: the k-th state is (2^N - 1) xor k with E = -(2^N-1) + 2k."""
    N = 22
    J, h = I.free_spins_pow2_fields(N)
    S = 3000
    m, e = gpu_search(torch_dev, J, h, S)
    k = np.arange(S)
    assert np.array_equal(m.astype(np.int64), ((1 << N) - 1) ^ k)
    assert np.array_equal(e.astype(np.int64), -((1 << N) - 1) + 2 * k)


@pytest.mark.parametrize("S,dtype", [(1, np.int32), (100, np.int32), (4095, np.int32),
                                     (100, np.float32)])
def test_pow2_fields_many_survivors(torch_dev, S, dtype):
    """J = 0, h_i = 2^i: energies fall with the mask, so every state of a later
    chunk beats the record and the merge receives whole chunks of survivors
    (far more than its LDS holds): it keeps only those at or below the S-th
    smallest survivor key.  Closed form as above."""
    N = 22
    J, h = I.free_spins_pow2_fields(N, dtype=dtype)
    m, e = gpu_search(torch_dev, J, h, S)
    k = np.arange(S)
    assert np.array_equal(m.astype(np.int64), ((1 << N) - 1) ^ k)
    assert np.array_equal(e.astype(np.int64), -((1 << N) - 1) + 2 * k)


def test_merge_ties_beyond_lds(torch_dev):
    """h_i = 2^i for spins 13..21 only: every energy is shared by the 8192
    masks of one setting of the top spins, and later chunks again beat the
    record, so the survivors at the S-th smallest key (8192 of them) exceed the
    merge's LDS and it sorts them all; the S lowest are the S smallest masks
    with every top spin up (ties go by mask)."""
    N, lo = 22, 13
    J = np.zeros((N, N), dtype=np.int32)
    h = np.zeros(N, dtype=np.int32)
    h[lo:] = 2 ** np.arange(lo, N)
    S = 100
    m, e = gpu_search(torch_dev, J, h, S)
    top = ((1 << (N - lo)) - 1) << lo
    assert np.array_equal(m.astype(np.int64), top | np.arange(S))
    assert np.all(e.astype(np.int64) == -int(h.sum()))


def test_prefix_monotone_and_deterministic(torch_dev):
    J, h = I.random_int_dense(26, 5)
    m1, e1 = gpu_search(torch_dev, J, h, 10)
    m2, e2 = gpu_search(torch_dev, J, h, 2000)
    m3, e3 = gpu_search(torch_dev, J, h, 2000)
    assert np.array_equal(m1, m2[:10]) and np.array_equal(e1, e2[:10])
    assert np.array_equal(m2, m3) and np.array_equal(e2, e3)


def test_device_errors(torch_dev):
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    J, h = I.random_f32_dense(12, 3)
    J[0, 5] = np.nan
    with pytest.raises(sg.SgError) as ei:
        gpu_search(torch_dev, J, h, 10)
    assert ei.value.status == _lib.SG_ENONFINITE
    Ji, hi = I.random_int_dense(12, 3)
    Ji[0, 1] = 1 << 28
    with pytest.raises(sg.SgError) as ei:
        gpu_search(torch_dev, Ji, hi, 10)
    assert ei.value.status == _lib.SG_EOVERFLOW
    # the stream is clean again afterwards
    J, h = I.random_int_dense(12, 3)
    m, e = gpu_search(torch_dev, J, h, 10)
    assert len(m) == 10


def test_validation_errors(torch_dev):
    import paper_1904_03621_amd as sg
    J, h = I.random_int_dense(8, 3)
    with pytest.raises(sg.SgError):
        gpu_search(torch_dev, J, h, 257)       # S > 2^N
    with pytest.raises(sg.SgError):
        gpu_search(torch_dev, J, h, 4, 10, 64)  # lo not 64-aligned


def test_maximum_S_single(orc, torch_dev):
    """S = SG_MAX_S (2^20) on the N = 24 integer workload: bit-exact."""
    J, h = I.random_int_dense(24, 1)
    compare(orc, torch_dev, J, h, 1 << 20, what="N=24 S=2^20")


@pytest.mark.parametrize("N,lo,hi", [
    (56, (1 << 55) + (3 << 40), (1 << 55) + (3 << 40) + (1 << 20)),
    (63, (1 << 63) - (1 << 20), 1 << 63),                  # SG_MAX_N, last masks
    (63, (1 << 62) + (5 << 44) + 64 * 12345, (1 << 62) + (5 << 44) + 64 * 12345 + 3000000),
])
def test_maximum_N_range(orc, torch_dev, N, lo, hi):
    """Large N through the range API, up to N = SG_MAX_N = 63 and the range end
    2^63: slices high in the space against the oracle on the same slice."""
    J, h = I.random_int_dense(N, N)
    compare(orc, torch_dev, J, h, 64, lo, hi, what="N=%d slice" % N)
    Jf, hf = I.random_f32_dense(N, N + 1)
    compare(orc, torch_dev, Jf, hf, 64, lo, hi, what="N=%d f32 slice" % N)


@pytest.mark.parametrize("N,S", [(8, 256), (12, 4096), (20, 500), (24, 300)])
def test_int32_walk_large_couplings(orc, torch_dev, N, S):
    """Integer couplings too large for the exact fp32 walk (2.1 sum|J| >= 2^24,
    below the 2^28 overflow bound): the int32 walk, bit-exact."""
    J, h = I.random_int_dense(N, 500 + N, lo=-(1 << 20), hi=1 << 20)
    bound = int(np.abs(np.triu(J.astype(np.int64), 1)).sum() + np.abs(h.astype(np.int64)).sum())
    assert 2.1 * bound >= (1 << 24) and bound < (1 << 28), bound
    compare(orc, torch_dev, J, h, S, what="int32 walk N=%d" % N)


def test_int_walk_boundary(orc, torch_dev):
    """Integer instances just below and just above the fp32-walk limit
    (2.1 sum|J| < 2^24 takes the fp32 walk): both bit-exact."""
    N = 16
    J0, h0 = I.random_int_dense(N, 77)
    b0 = int(np.abs(np.triu(J0.astype(np.int64), 1)).sum() + np.abs(h0.astype(np.int64)).sum())
    for target in ((1 << 24) / 2.1 - 64, (1 << 24) / 2.1 + 64):
        k = int(target // b0)
        J, h = (J0.astype(np.int64) * k).astype(np.int32), (h0.astype(np.int64) * k).astype(np.int32)
        compare(orc, torch_dev, J, h, 1000, what="int walk limit x%d" % k)


def test_every_state_at_block_boundaries(orc, torch_dev):
    """N = 7 and 8 (one and two 128-state blocks): every state, both paths."""
    for N in (7, 8):
        J, h = I.random_int_dense(N, 300 + N)
        compare(orc, torch_dev, J, h, 1 << N, what="int N=%d all" % N)
        Jf, hf = I.random_f32_dense(N, 310 + N, j_scale=1.0, h_scale=0.3)
        compare(orc, torch_dev, Jf, hf, 1 << N, what="f32 N=%d all" % N)
