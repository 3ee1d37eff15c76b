"""log Z(beta) forward and backward on the GPU against the CPU oracle, closed
forms and central finite differences; the 256 x N = 28 workload shape checked
on a sampled instance and through the identity that ties the gradients to the
beta-derivative of log Z.

Tolerances: log Z within 1e-6 relative; gradients within 1e-5 of the largest
gradient entry of the instance (element-wise relative error is meaningless for
entries that vanish)."""

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


def to_dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def gpu_forward(torch, J, h, betas, S):
    import paper_1904_03621_amd as sg
    Jt, ht, bt = to_dev(torch, J, h, np.asarray(betas, dtype=np.float32))
    lz, e0, m, e = sg.logz_forward(Jt, ht, bt, S)
    return lz.cpu().numpy(), e0.cpu().numpy(), m.cpu().numpy().astype(np.uint64), e.cpu().numpy()


def gpu_backward(torch, J, h, betas, g, S=1):
    import paper_1904_03621_amd as sg
    Jt, ht, bt = to_dev(torch, J, h, np.asarray(betas, dtype=np.float32))
    lz, e0, _, _ = sg.logz_forward(Jt, ht, bt, S)
    gt = torch.from_numpy(np.asarray(g, dtype=np.float64)).cuda()
    gJ, gh = sg.logz_backward(Jt, ht, bt, e0, lz, gt)
    return gJ.cpu().numpy().astype(np.float64), gh.cpu().numpy().astype(np.float64)


def check_logz(lz, lz_ref, what):
    err = np.abs(lz - lz_ref) / np.maximum(np.abs(lz_ref), 1e-300)
    assert np.all(err <= 1e-6), "%s: log Z rel err %.3g\n%s\n%s" % (what, err.max(), lz, lz_ref)


def check_grad(gJ, gh, gJ_ref, gh_ref, what):
    N = len(gh)
    iu = np.triu_indices(N, 1)
    scale = max(np.abs(gJ_ref[iu]).max() if N > 1 else 0.0, np.abs(gh_ref).max(), 1e-30)
    eJ = np.abs(gJ[iu] - gJ_ref[iu]).max() / scale if N > 1 else 0.0
    eh = np.abs(gh - gh_ref).max() / scale
    assert eJ <= 1e-5 and eh <= 1e-5, "%s: grad err J %.3g h %.3g" % (what, eJ, eh)
    low = np.tril_indices(N)
    assert np.all(gJ[low] == 0.0), "%s: grad_J nonzero on or below the diagonal" % what


@pytest.mark.parametrize("N", [7, 8, 9, 10, 11, 13, 14, 15, 17, 20])
def test_forward_backward_vs_oracle(orc, torch_dev, N):
    """Three instances, three beta: the partition sums over blocks of 6
    (N = 7), 8 (N = 8, 9) and 10 (one record per lane at N = 10, two at 11),
    the gradient walk over blocks of 6 and records of 8."""
    B = 3
    J, h = I.logz_batch(B, N, 40 + N)
    S = min(32, 1 << N)
    lz, e0, m, e = gpu_forward(torch_dev, J, h, BETAS, S)
    rng = np.random.default_rng(N)
    g = rng.standard_normal((B, len(BETAS)))
    gJ, gh = gpu_backward(torch_dev, J, h, BETAS, g, S)
    for b in range(B):
        lz_ref, e0_ref = orc.logz(J[b], h[b], BETAS)
        check_logz(lz[b], lz_ref, "N=%d b=%d" % (N, b))
        tau = 1e-5 * np.abs(np.triu(J[b].astype(np.float64), 1)).sum()
        assert abs(e0[b] - e0_ref) <= tau and e0[b] == e[b, 0]
        om, oe = orc.low_spectrum(J[b], h[b], S)
        assert np.all(np.abs(e[b].astype(np.float64) - oe) <= tau)
        gJ_ref, gh_ref = orc.logz_grad(J[b], h[b], BETAS, g[b])
        check_grad(gJ[b], gh[b], gJ_ref, gh_ref, "N=%d b=%d" % (N, b))


@pytest.mark.parametrize("betas", [[1.3], [0.25, 3.0], [0.2, 0.7, 1.5, 2.5]])
@pytest.mark.parametrize("N", [7, 12])
def test_beta_counts_vs_oracle(orc, torch_dev, N, betas):
    """One, two and four inverse temperatures (each count is its own kernel):
    the partition sums over blocks of 6 low spins (N = 7), of 10 (N = 12, one
    and two beta) and of 8 (N = 12, four beta); the gradient walk over blocks
    of 6 (N = 7) and records of 8 (N = 12)."""
    B = 2
    J, h = I.logz_batch(B, N, 60 + N + len(betas))
    lz, _, _, _ = gpu_forward(torch_dev, J, h, betas, 8)
    rng = np.random.default_rng(100 + N + len(betas))
    g = rng.standard_normal((B, len(betas)))
    gJ, gh = gpu_backward(torch_dev, J, h, betas, g)
    for b in range(B):
        what = "N=%d nb=%d b=%d" % (N, len(betas), b)
        check_logz(lz[b], orc.logz(J[b], h[b], betas)[0], what)
        gJ_ref, gh_ref = orc.logz_grad(J[b], h[b], betas, g[b])
        check_grad(gJ[b], gh[b], gJ_ref, gh_ref, what)


def test_states_match_batched_search(torch_dev):
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, N, S = 16, 18, 32
    J, h = I.logz_batch(B, N, 7)
    _, _, m, e = gpu_forward(torch, J, h, BETAS, S)
    Ns = np.full(B, N, dtype=np.int32)
    bm, be = sg.low_spectrum_batched(*to_dev(torch, Ns, J, h), S)
    assert np.array_equal(m, bm.cpu().numpy().astype(np.uint64))
    assert np.array_equal(e, be.cpu().numpy())


def test_n22_batch(orc, torch_dev):
    B, N = 2, 22
    J, h = I.logz_batch(B, N, 22)
    g = np.array([[1.0, -0.5, 0.25], [0.0, 1.0, 0.0]])
    lz, _, _, _ = gpu_forward(torch_dev, J, h, BETAS, 32)
    gJ, gh = gpu_backward(torch_dev, J, h, BETAS, g)
    for b in range(B):
        check_logz(lz[b], orc.logz(J[b], h[b], BETAS)[0], "N=22 b=%d" % b)
        gJ_ref, gh_ref = orc.logz_grad(J[b], h[b], BETAS, g[b])
        check_grad(gJ[b], gh[b], gJ_ref, gh_ref, "N=22 b=%d" % b)


def test_free_spins_closed_form(torch_dev):
    """J = 0: log Z = sum_i log(2 cosh(beta h_i)), <s_i> = tanh(beta h_i),
    <s_i s_j> = tanh(beta h_i) tanh(beta h_j)."""
    B, N = 2, 16
    rng = np.random.default_rng(3)
    J = np.zeros((B, N, N), dtype=np.float32)
    h = (rng.standard_normal((B, N)) * 0.5).astype(np.float32)
    lz, e0, _, _ = gpu_forward(torch_dev, J, h, BETAS, 8)
    g = np.zeros((B, 3))
    g[:, 1] = 1.0  # beta = 1
    gJ, gh = gpu_backward(torch_dev, J, h, BETAS, g)
    hd = h.astype(np.float64)
    for b in range(B):
        want = [np.sum(np.log(2.0 * np.cosh(bt * hd[b]))) for bt in BETAS]
        check_logz(lz[b], np.array(want), "free b=%d" % b)
        assert abs(e0[b] + np.abs(hd[b]).sum()) <= 1e-5
        t = np.tanh(hd[b])
        check_grad(gJ[b], gh[b], np.triu(np.outer(t, t), 1), t, "free b=%d" % b)


def test_free_spins_closed_form_n36(torch_dev):
    """J = 0 at N = 36 (2^36 states, beyond the oracle): log Z, <s_i> and
    <s_i s_j> in closed form."""
    N = 36
    rng = np.random.default_rng(31)
    J = np.zeros((1, N, N), dtype=np.float32)
    h = (rng.standard_normal((1, N)) * 0.5).astype(np.float32)
    lz, _, _, _ = gpu_forward(torch_dev, J, h, BETAS, 8)
    g = np.array([[0.0, 1.0, 0.0]])
    gJ, gh = gpu_backward(torch_dev, J, h, BETAS, g)
    hd = h[0].astype(np.float64)
    check_logz(lz[0], np.array([np.sum(np.log(2.0 * np.cosh(bt * hd))) for bt in BETAS]),
               "free N=36")
    t = np.tanh(hd)
    check_grad(gJ[0], gh[0], np.triu(np.outer(t, t), 1), t, "free N=36")


def test_open_chain_n40_closed_form(torch_dev):
    """Open chain of 40 spins, h = 0: Z = 2 prod_i 2 cosh(beta K_i) and
    <s_i s_j> = prod_{i <= l < j} tanh(beta K_l) (2^40 states)."""
    N = 40
    rng = np.random.default_rng(41)
    K = (rng.standard_normal(N - 1) * 0.8).astype(np.float32)
    J = np.zeros((1, N, N), dtype=np.float32)
    for i in range(N - 1):
        J[0, i, i + 1] = K[i]
    h = np.zeros((1, N), dtype=np.float32)
    lz, _, _, _ = gpu_forward(torch_dev, J, h, BETAS, 4)
    Kd = K.astype(np.float64)
    want = [np.log(2.0) + np.sum(np.log(2.0 * np.cosh(bt * Kd))) for bt in BETAS]
    check_logz(lz[0], np.array(want), "chain N=40")
    g = np.array([[0.0, 1.0, 0.0]])  # beta = 1
    gJ, gh = gpu_backward(torch_dev, J, h, BETAS, g)
    t = np.tanh(Kd)
    ref = np.zeros((N, N))
    for i in range(N):
        prod = 1.0
        for j in range(i + 1, N):
            prod *= t[j - 1]
            ref[i, j] = prod
    check_grad(gJ[0], gh[0], ref, np.zeros(N), "chain N=40")


def test_open_chain_transfer_matrix(torch_dev):
    """Open chain (J_{i,i+1} only): log Z from 2 x 2 transfer matrices."""
    N = 20
    rng = np.random.default_rng(9)
    J = np.zeros((1, N, N), dtype=np.float32)
    for i in range(N - 1):
        J[0, i, i + 1] = rng.standard_normal()
    h = (rng.standard_normal((1, N)) * 0.3).astype(np.float32)
    lz, _, _, _ = gpu_forward(torch_dev, J, h, BETAS, 4)
    Jd, hd = J[0].astype(np.float64), h[0].astype(np.float64)
    sv = np.array([-1.0, 1.0])
    for k, bt in enumerate(BETAS):
        v = np.exp(bt * hd[0] * sv)
        logscale = 0.0
        for i in range(1, N):
            M = np.exp(bt * Jd[i - 1, i] * np.outer(sv, sv) + bt * hd[i] * sv[None, :])
            v = v @ M
            c = v.max()
            v /= c
            logscale += np.log(c)
        want = logscale + np.log(v.sum())
        check_logz(lz[0, k:k + 1], np.array([want]), "chain beta=%g" % bt)


def test_gradient_vs_central_differences(orc, torch_dev):
    """GPU gradient against central differences of the oracle's log Z."""
    B, N = 1, 10
    J, h = I.logz_batch(B, N, 17)
    g = np.array([[0.3, 1.0, -0.7]])
    gJ, gh = gpu_backward(torch_dev, J, h, BETAS, g)
    Jd, hd = J[0].astype(np.float64), h[0].astype(np.float64)

    def f(Jx, hx):
        return float(np.dot(g[0], orc.logz(Jx, hx, BETAS)[0]))

    d = 1e-4
    for (i, j) in [(0, 1), (2, 7), (8, 9), (0, 9)]:
        Jp, Jm = Jd.copy(), Jd.copy()
        Jp[i, j] += d
        Jm[i, j] -= d
        fd = (f(Jp, hd) - f(Jm, hd)) / (2 * d)
        assert abs(gJ[0, i, j] - fd) <= 1e-5 * max(1.0, abs(fd)), (i, j, gJ[0, i, j], fd)
    for i in [0, 4, 9]:
        hp, hm = hd.copy(), hd.copy()
        hp[i] += d
        hm[i] -= d
        fd = (f(Jd, hp) - f(Jd, hm)) / (2 * d)
        assert abs(gh[0, i] - fd) <= 1e-5 * max(1.0, abs(fd)), (i, gh[0, i], fd)


def test_autograd_function(orc, torch_dev):
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, N = 2, 12
    J, h = I.logz_batch(B, N, 5)
    Jt, ht, bt = to_dev(torch, J, h, np.asarray(BETAS, dtype=np.float32))
    Jt.requires_grad_(True)
    ht.requires_grad_(True)
    w = torch.tensor([[1.0, 2.0, -1.0], [0.5, 0.0, 1.5]], dtype=torch.float64, device="cuda")
    lz, states, energies = sg.logz(Jt, ht, bt, 16)
    assert lz.requires_grad and not states.requires_grad and not energies.requires_grad
    (lz * w).sum().backward()
    wn = w.cpu().numpy()
    for b in range(B):
        gJ_ref, gh_ref = orc.logz_grad(J[b], h[b], BETAS, wn[b])
        check_grad(Jt.grad[b].cpu().numpy().astype(np.float64),
                   ht.grad[b].cpu().numpy().astype(np.float64), gJ_ref, gh_ref, "autograd %d" % b)


def test_workload_shape(orc, torch_dev):
    """256 instances, N = 28, beta in {0.5, 1, 2}, S = 32.  Instance 0's log Z
    against the oracle; for every instance, sum_{i<j} J_ij dlogZ/dJ_ij +
    sum_i h_i dlogZ/dh_i = -beta <E> = beta dlogZ/dbeta, the beta-derivative
    taken by central differences of the GPU forward."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, N, S = 256, 28, 32
    J, h = I.logz_batch(B, N, 2028)
    Jt, ht = to_dev(torch, J, h)
    bt = torch.tensor(BETAS, dtype=torch.float32, device="cuda")
    lz, e0, m, e = sg.logz_forward(Jt, ht, bt, S)
    lz = lz.cpu().numpy()
    check_logz(lz[0], orc.logz(J[0], h[0], BETAS)[0], "N=28 b=0")
    om, oe = orc.low_spectrum(J[0], h[0], S)
    tau = 1e-5 * np.abs(J[0].astype(np.float64)).sum()
    assert np.all(np.abs(e[0].cpu().numpy().astype(np.float64) - oe) <= tau)
    k = 1  # beta = 1
    g = torch.zeros((B, 3), dtype=torch.float64, device="cuda")
    g[:, k] = 1.0
    gJ, gh = sg.logz_backward(Jt, ht, bt, e0, torch.from_numpy(lz).cuda(), g)
    lhs = ((gJ.double() * Jt.double()).sum(dim=(1, 2)) + (gh.double() * ht.double()).sum(dim=1))
    lhs = lhs.cpu().numpy() / BETAS[k]
    d = 1e-3
    bpm = torch.tensor([BETAS[k] + d, BETAS[k] - d], dtype=torch.float32, device="cuda")
    lzpm, _, _, _ = sg.logz_forward(Jt, ht, bpm, S)
    lzpm = lzpm.cpu().numpy()
    db = float(bpm[0].item()) - float(bpm[1].item())
    fd = (lzpm[:, 0] - lzpm[:, 1]) / db
    err = np.abs(lhs - fd) / np.maximum(np.abs(fd), 1.0)
    assert err.max() <= 1e-4, err.max()


def test_errors(torch_dev):
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    torch = torch_dev
    J, h = I.logz_batch(2, 10, 1)
    Jt, ht = to_dev(torch, J, h)
    with pytest.raises(sg.SgError) as ei:
        sg.logz_forward(Jt, ht, torch.tensor([1.0, -1.0], device="cuda"), 4)
    assert ei.value.status == _lib.SG_EINVAL
    with pytest.raises(sg.SgError) as ei:
        sg.logz_forward(Jt, ht, torch.ones(5, device="cuda"), 4)
    assert ei.value.status == _lib.SG_EINVAL
    J6, h6 = I.logz_batch(1, 6, 1)
    with pytest.raises(sg.SgError) as ei:
        sg.logz_forward(*to_dev(torch, J6, h6), torch.ones(1, device="cuda"), 4)
    assert ei.value.status == _lib.SG_EINVAL
    # the stream is clean again
    lz, e0, _, _ = sg.logz_forward(Jt, ht, torch.ones(1, device="cuda"), 4)
    assert np.all(np.isfinite(lz.cpu().numpy()))
    # a NaN coupling handed to the backward alone is reported too
    Jn = J.copy()
    Jn[1, 2, 5] = np.nan
    with pytest.raises(sg.SgError) as ei:
        sg.logz_backward(to_dev(torch, Jn)[0], ht, torch.ones(1, device="cuda"), e0, lz,
                         torch.ones((2, 1), dtype=torch.float64, device="cuda"))
    assert ei.value.status == _lib.SG_ENONFINITE


def test_gauge_and_permutation_invariance_n32(torch_dev):
    """Beyond the oracle's reach (N = 32): a gauge transform J'_ij = t_i t_j J_ij,
    h'_i = t_i h_i (t_i = +-1) and a relabelling of the spins leave log Z
    unchanged and map the gradients the same way."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, N = 2, 32
    J, h = I.logz_batch(B, N, 32)
    rng = np.random.default_rng(5)
    t = rng.choice(np.array([-1.0, 1.0]), size=(B, N))
    perm = np.stack([rng.permutation(N) for _ in range(B)])
    Jg = np.zeros_like(J)
    hg = np.zeros_like(h)
    for b in range(B):
        full = J[b].astype(np.float64) + J[b].astype(np.float64).T
        fg = full * np.outer(t[b], t[b])
        fp = fg[np.ix_(perm[b], perm[b])]
        Jg[b] = np.triu(fp, 1).astype(np.float32)
        hg[b] = (h[b] * t[b])[perm[b]].astype(np.float32)
    g = np.array([[1.0, -0.5, 0.25], [0.3, 0.3, 0.3]])
    lz, _, _, _ = gpu_forward(torch, J, h, BETAS, 16)
    lz2, _, _, _ = gpu_forward(torch, Jg, hg, BETAS, 16)
    assert np.all(np.abs(lz - lz2) <= 1e-6 * np.abs(lz)), (lz, lz2)
    gJ, gh = gpu_backward(torch, J, h, BETAS, g)
    gJ2, gh2 = gpu_backward(torch, Jg, hg, BETAS, g)
    for b in range(B):
        # map the transformed gradients back to the original labels and signs
        fullg2 = gJ2[b] + gJ2[b].T
        back = np.zeros((N, N))
        back[np.ix_(perm[b], perm[b])] = fullg2
        back *= np.outer(t[b], t[b])
        hb = np.zeros(N)
        hb[perm[b]] = gh2[b]
        hb *= t[b]
        check_grad(np.triu(back, 1), hb, gJ[b], gh[b], "gauge/permutation b=%d" % b)
