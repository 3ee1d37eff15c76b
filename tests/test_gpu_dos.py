"""Density of states on the GPU: bit for bit against the CPU oracle at sizes it
finishes in seconds, against closed forms and invariants at N = 40, and
against the low-spectrum search at the bottom of the spectrum."""

import math

import numpy as np
import pytest

import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def gpu_dos(torch, J, h, e_min=None, n_bins=None):
    import paper_1904_03621_amd as sg
    Jt = torch.from_numpy(np.ascontiguousarray(J, dtype=np.int32)).cuda()
    ht = torch.from_numpy(np.ascontiguousarray(h, dtype=np.int32)).cuda()
    e0, counts = sg.density_of_states(Jt, ht, e_min, n_bins)
    return e0, counts.cpu().numpy().astype(np.uint64)


@pytest.mark.parametrize("N,seed", [(1, 1), (3, 2), (6, 3), (7, 4), (8, 5), (11, 6), (16, 7),
                                    (20, 8), (22, 9)])
def test_vs_oracle(orc, torch_dev, N, seed):
    J, h = I.random_int_dense(N, seed)
    e0, counts = gpu_dos(torch_dev, J, h)
    oe0, ocounts = orc.density_of_states(J, h)
    assert e0 == oe0
    assert np.array_equal(counts, ocounts), "N=%d" % N
    assert int(counts.sum()) == 1 << N


def test_chimera_small_vs_oracle(orc, torch_dev):
    J, h = I.chimera_pm1(1, 3, 21)  # 24 spins
    e0, counts = gpu_dos(torch_dev, J, h)
    oe0, ocounts = orc.density_of_states(J, h)
    assert e0 == oe0 and np.array_equal(counts, ocounts)


def test_ferromagnet_n40_closed_form(torch_dev):
    """J = 1 on the complete graph, N = 40: C(40, c) states at
    E = -((40 - 2c)^2 - 40) / 2 for each popcount c; all 2^40 enumerated."""
    N = 40
    J, h = I.ferromagnet(N, 1, np.int32)
    e0, counts = gpu_dos(torch_dev, J, h)
    want = np.zeros_like(counts)
    for c in range(N + 1):
        want[-((N - 2 * c) ** 2 - N) // 2 - e0] += math.comb(N, c)
    assert np.array_equal(counts, want)


def test_chimera_n40_invariants_and_search(torch_dev):
    """Chimera 1 x 5 cells (40 spins), couplers +-1, h = 0: every level holds an
    even number of states (global flip), the counts sum to 2^40, and the bottom
    of the spectrum agrees with the low-spectrum search."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    J, h = I.chimera_pm1(1, 5, 6)
    e0, counts = gpu_dos(torch, J, h)
    assert int(counts.sum()) == 1 << 40
    assert np.all(counts % 2 == 0)
    S = 5000
    m, e = sg.low_spectrum(torch.from_numpy(J).cuda(), torch.from_numpy(h).cuda(), S)
    e = e.cpu().numpy().astype(np.int64)
    top = e[-1]
    vals, cnt = np.unique(e[e < top], return_counts=True)
    for v, c in zip(vals, cnt):
        assert counts[v - e0] == c, (v, c, counts[v - e0])
    assert counts[top - e0] >= np.sum(e == top)
    assert np.all(counts[:e[0] - e0] == 0)


def test_custom_bins_and_errors(orc, torch_dev):
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    torch = torch_dev
    J, h = I.random_int_dense(12, 3)
    B = orc.energy_bound(J, h)
    # wider bins than needed: the same counts, shifted
    e0, counts = gpu_dos(torch, J, h, -B - 5, 2 * B + 20)
    oe0, ocounts = orc.density_of_states(J, h)
    assert np.array_equal(counts[5:5 + len(ocounts)], ocounts) and counts[:5].sum() == 0
    # bins that do not cover [-B, B]: reported, counts zero
    with pytest.raises(sg.SgError) as ei:
        gpu_dos(torch, J, h, -B + 1, 2 * B + 1)
    assert ei.value.status == _lib.SG_EINVAL
    Jb = J.copy()
    Jb[0, 1] = 1 << 28
    with pytest.raises(sg.SgError) as ei:
        gpu_dos(torch, Jb, h, -10, 21)
    assert ei.value.status in (_lib.SG_EOVERFLOW, _lib.SG_EINVAL)
    # the stream is clean again
    e0, counts = gpu_dos(torch, J, h)
    assert int(counts.sum()) == 1 << 12
