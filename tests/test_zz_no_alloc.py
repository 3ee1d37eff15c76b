"""The allocation-free log Z backward (sg_logz_backward_noalloc_f32), called
through the C ABI, against the allocating entry point sg_logz_backward_f32 on
the same inputs and stream: two calls in a row, the second smaller (the
static scratch keeps the first call's contents), then the size limit, the
device error word and a clean call after it.

Tolerance: gradients within 1e-5 of the largest gradient entry of the
instance, as for the backward against the oracle (both entry points run the
same kernels; only the order of the fp64 atomic adds may differ)."""

import numpy as np
import pytest

import instances as I

pytestmark = pytest.mark.gpu

BETAS = [0.5, 1.0, 2.0]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def _inputs(torch, B, N, betas, seed):
    import paper_1904_03621_amd as sg
    J, h = I.logz_batch(B, N, seed)
    Jt = torch.from_numpy(np.ascontiguousarray(J)).cuda()
    ht = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    bt = torch.tensor(betas, dtype=torch.float32, device="cuda")
    lz, e0, _, _ = sg.logz_forward(Jt, ht, bt, 1)
    rng = np.random.default_rng(seed)
    g = torch.from_numpy(rng.uniform(-1.0, 1.0, size=(B, len(betas)))).cuda()
    return Jt, ht, bt, e0, lz, g


def _call(torch, fn, B, N, K, Jt, ht, bt, e0, lz, g):
    from paper_1904_03621_amd import _lib
    # outputs start as NaN: every entry must be written by the call
    gJ = torch.full((B, N, N), float("nan"), dtype=torch.float32, device="cuda")
    gh = torch.full((B, N), float("nan"), dtype=torch.float32, device="cuda")
    st = fn(B, N, Jt, ht, K, bt, e0, lz, g, gJ, gh)
    _lib.check(st, fn.__name__)
    _lib.check(_lib.sg_get_error(), "device")
    return gJ.cpu().numpy().astype(np.float64), gh.cpu().numpy().astype(np.float64)


def _check(a, b, what):
    aJ, ah = a
    bJ, bh = b
    B, N = ah.shape
    iu = np.triu_indices(N, 1)
    low = np.tril_indices(N)
    for i in range(B):
        assert np.all(np.isfinite(aJ[i])) and np.all(np.isfinite(ah[i])), what
        scale = max(np.abs(bJ[i][iu]).max(), np.abs(bh[i]).max(), 1e-30)
        eJ = np.abs(aJ[i][iu] - bJ[i][iu]).max() / scale
        eh = np.abs(ah[i] - bh[i]).max() / scale
        assert eJ <= 1e-5 and eh <= 1e-5, "%s instance %d: err J %.3g h %.3g" % (what, i, eJ, eh)
        assert np.all(aJ[i][low] == 0.0), "%s: grad_J nonzero on or below the diagonal" % what


@pytest.mark.parametrize("first, second", [
    ((256, 28, BETAS), (16, 14, [0.7, 1.3])),   # records of 8 with 6 high spins, then fewer
    ((64, 20, [1.0]), (3, 7, BETAS)),           # then N = 7 (blocks of 6)
])
def test_noalloc_matches_allocating_entry(torch_dev, first, second):
    from paper_1904_03621_amd import _lib
    torch = torch_dev
    for k, (B, N, betas) in enumerate((first, second)):
        print("noalloc parity: call %d B=%d N=%d betas=%s" % (k, B, N, betas), flush=True)
        args = _inputs(torch, B, N, betas, 300 + 7 * N + B)
        ref = _call(torch, _lib.sg_logz_backward_f32, B, N, len(betas), *args)
        got = _call(torch, _lib.sg_logz_backward_noalloc_f32, B, N, len(betas), *args)
        _check(got, ref, "B=%d N=%d" % (B, N))


def test_noalloc_limit_and_errors(torch_dev):
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    torch = torch_dev
    lib = _lib.lib()
    # more than the static scratch holds: refused before any work is enqueued
    B, N = 2048, 28
    p = 4096  # never dereferenced: the size check fails first
    st = lib.sg_logz_backward_noalloc_f32(B, N, p, p, 3, p, p, p, p, p, p, 0)
    assert st == _lib.SG_EINVAL
    assert "SG_LOGZ_SCRATCH_BYTES" in _lib.last_error()
    # a NaN coupling is reported through the scratch's error word ...
    J, h = I.logz_batch(2, 10, 1)
    Jt = torch.from_numpy(np.ascontiguousarray(J)).cuda()
    ht = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    one = torch.ones(1, device="cuda")
    lz, e0, _, _ = sg.logz_forward(Jt, ht, one, 4)
    gl = torch.ones((2, 1), dtype=torch.float64, device="cuda")
    Jn = J.copy()
    Jn[1, 2, 5] = np.nan
    Jnt = torch.from_numpy(Jn).cuda()
    with pytest.raises(sg.SgError) as ei:
        sg.logz_backward(Jnt, ht, one, e0, lz, gl, no_alloc=True)
    assert ei.value.status == _lib.SG_ENONFINITE
    # ... and cleared by reading it: the next call is clean
    gJ, gh = sg.logz_backward(Jt, ht, one, e0, lz, gl, no_alloc=True)
    rJ, rh = sg.logz_backward(Jt, ht, one, e0, lz, gl)
    _check((gJ.cpu().numpy().astype(np.float64), gh.cpu().numpy().astype(np.float64)),
           (rJ.cpu().numpy().astype(np.float64), rh.cpu().numpy().astype(np.float64)), "clean")
