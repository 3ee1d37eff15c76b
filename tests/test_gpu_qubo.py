"""QUBO front end (Eqs. 2-3) on the GPU: against the Ising search of the
instance it comes from (same states, energies shifted by the offset of Eq. 3)
and against brute force over the QUBO form of the oracle."""

import numpy as np
import pytest

import instances as I
from parity import check_f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def gpu_qubo(torch, a, b, S):
    import paper_1904_03621_amd as sg
    A = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    bt = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).cuda()
    m, e = sg.low_spectrum_qubo(A, bt, S)
    return m.cpu().numpy().astype(np.uint64), e.cpu().numpy()


def brute_force(orc, a, b):
    N = len(b)
    f = np.array([orc.qubo_energy(a, b, m) for m in range(1 << N)])
    order = np.lexsort((np.arange(1 << N), f))
    return order.astype(np.uint64), f[order]


@pytest.mark.parametrize("N,seed", [(4, 1), (9, 2), (20, 3)])
def test_matches_ising_search(orc, torch_dev, N, seed):
    """An integer Ising instance and its QUBO form: the same states in the same
    order, F = H - (sum h - sum J) exactly."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    J, h = I.random_int_dense(N, seed)
    a, b, off = orc.qubo_from_ising(J, h)
    S = min(200, 1 << N)
    qm, qe = gpu_qubo(torch, a, b, S)
    im, ie = sg.low_spectrum(torch.from_numpy(J).cuda(), torch.from_numpy(h).cuda(), S)
    im = im.cpu().numpy().astype(np.uint64)
    ie = ie.cpu().numpy().astype(np.int64)
    assert np.array_equal(qm, im)
    assert np.array_equal(qe.astype(np.float64), (ie - off).astype(np.float64))


def test_brute_force_integer(orc, torch_dev):
    rng = np.random.default_rng(7)
    N = 12
    a = np.triu(rng.integers(-5, 6, size=(N, N)), 1).astype(np.float32)
    b = rng.integers(-5, 6, size=N).astype(np.float32)
    om, oe = brute_force(orc, a, b)
    m, e = gpu_qubo(torch_dev, a, b, 300)
    assert np.array_equal(m, om[:300]) and np.array_equal(e.astype(np.float64), oe[:300])


def test_brute_force_float(orc, torch_dev):
    rng = np.random.default_rng(8)
    N = 13
    a = np.triu(rng.standard_normal((N, N)), 1).astype(np.float32)
    b = rng.standard_normal(N).astype(np.float32)
    om, oe = brute_force(orc, a, b)
    S = 500
    m, e = gpu_qubo(torch_dev, a, b, S)
    # the tolerance rules of the fp32 search, with the QUBO couplings in J's place
    check_f32(N, a, m, e, om[:S], oe[:S], lambda x: orc.qubo_energy(a, b, x), "qubo N=13")


def test_validation(torch_dev):
    import paper_1904_03621_amd as sg
    with pytest.raises(sg.SgError):
        gpu_qubo(torch_dev, np.zeros((3, 3)), np.zeros(3), 9)  # S > 2^N
