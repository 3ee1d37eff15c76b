"""Batched search: every instance of a batch against the CPU oracle and bit for
bit against the single-instance search, at small sizes, at the 4096-instance
workload shape, and replayed from a captured HIP graph."""

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


def make_batch(B, lo, hi, seed, isint, Nmax=None):
    rng = np.random.default_rng(seed)
    Ns = rng.integers(lo, hi + 1, size=B).astype(np.int32)
    Nmax = Nmax or hi
    dt = np.int32 if isint else np.float32
    J = np.zeros((B, Nmax, Nmax), dtype=dt)
    h = np.zeros((B, Nmax), dtype=dt)
    for b in range(B):
        n = int(Ns[b])
        if isint:
            Jb, hb = I.random_int_dense(n, 1000 + seed * 7919 + b)
        else:
            Jb, hb = I.random_f32_dense(n, 1000 + seed * 7919 + b, j_scale=1.0, h_scale=0.1)
        J[b, :n, :n] = Jb
        h[b, :n] = hb
    return Ns, J, h


def run_batched(torch, Ns, J, h, S):
    import paper_1904_03621_amd as sg
    m, e = sg.low_spectrum_batched(torch.from_numpy(Ns).cuda(), torch.from_numpy(J).cuda(),
                                   torch.from_numpy(h).cuda(), S)
    return m.cpu().numpy().astype(np.uint64), e.cpu().numpy()


def run_single(torch, J, h, S):
    import paper_1904_03621_amd as sg
    m, e = sg.low_spectrum(torch.from_numpy(np.ascontiguousarray(J)).cuda(),
                           torch.from_numpy(np.ascontiguousarray(h)).cuda(), S)
    return m.cpu().numpy().astype(np.uint64), e.cpu().numpy()


@pytest.mark.parametrize("isint", [True, False])
def test_small_batch_vs_oracle_and_single(orc, torch_dev, isint):
    B, S = 40, 32
    Ns, J, h = make_batch(B, 7, 20, 3, isint)
    bm, be = run_batched(torch_dev, Ns, J, h, S)
    for b in range(B):
        n = int(Ns[b])
        Jb, hb = J[b, :n, :n], h[b, :n]
        S_b = min(S, 1 << n)
        om, oe = orc.low_spectrum(Jb, hb, S_b)
        if isint:
            check_int(bm[b, :S_b], be[b, :S_b], om, oe, "batch %d (N=%d)" % (b, n))
        else:
            check_f32(n, Jb, bm[b, :S_b], be[b, :S_b], om, oe,
                      lambda x: orc.energy(Jb, hb, x), "batch %d (N=%d)" % (b, n))
        sm, se = run_single(torch_dev, Jb, hb, S_b)
        assert np.array_equal(sm, bm[b, :S_b]) and np.array_equal(se, be[b, :S_b])


def test_int_batch_mixes_both_walks(orc, torch_dev):
    """A batch of integer instances where every other one is scaled beyond the
    fp32-walk limit: both walks in the same launches, bit-exact per instance."""
    B, S = 24, 40
    Ns, J, h = make_batch(B, 8, 18, 11, True)
    J = J.astype(np.int64)
    h = h.astype(np.int64)
    J[1::2] *= 1 << 17
    h[1::2] *= 1 << 17
    J, h = J.astype(np.int32), h.astype(np.int32)
    bm, be = run_batched(torch_dev, Ns, J, h, S)
    for b in range(B):
        n = int(Ns[b])
        om, oe = orc.low_spectrum(J[b, :n, :n], h[b, :n], S)
        check_int(bm[b], be[b], om, oe, "batch %d (N=%d)" % (b, n))


def test_workload_shape_matches_single(orc, torch_dev):
    """N uniform in [16, 26] (the 4096-instance workload's distribution, cut at
    26 to keep the per-instance loop short), fp32, unscaled couplings, S = 64."""
    B, S = 256, 64
    Ns, J, h = make_batch(B, 16, 26, 4, False, Nmax=32)
    bm, be = run_batched(torch_dev, Ns, J, h, S)
    for b in range(B):
        n = int(Ns[b])
        sm, se = run_single(torch_dev, J[b, :n, :n], h[b, :n], S)
        assert np.array_equal(sm, bm[b]) and np.array_equal(se, be[b]), "instance %d" % b
    for b in range(0, B, 37):
        n = int(Ns[b])
        om, oe = orc.low_spectrum(J[b, :n, :n], h[b, :n], S)
        check_f32(n, J[b, :n, :n], bm[b], be[b], om, oe,
                  lambda x: orc.energy(J[b, :n, :n], h[b, :n], x), "oracle %d" % b)


def test_graph_replay(torch_dev):
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, S = 64, 16
    Ns, J, h = make_batch(B, 10, 22, 5, False)
    Nt, Jt, ht = (torch.from_numpy(x).cuda() for x in (Ns, J, h))
    m0, e0 = sg.low_spectrum_batched(Nt, Jt, ht, S)  # eager: sizes the workspace
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        m_out = torch.empty((B, S), dtype=torch.int64, device="cuda")
        e_out = torch.empty((B, S), dtype=torch.float32, device="cuda")
        sg.low_spectrum_batched(Nt, Jt, ht, S)  # same stream, eager, before capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            st = sg.sg_low_spectrum_batched_f32(B, Nt, J.shape[1], Jt, ht, S, m_out, e_out,
                                                stream)
        assert st == 0
    for rep in range(3):
        m_out.fill_(0)
        e_out.fill_(0)
        _ = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(m_out, m0) and torch.equal(e_out, e0), "replay %d differs" % rep
    assert sg.sg_get_error(stream) == 0


def test_bad_instance_size_reported(torch_dev):
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    Ns, J, h = make_batch(4, 8, 12, 6, True)
    Ns[2] = 6  # below 7
    with pytest.raises(sg.SgError) as ei:
        run_batched(torch_dev, Ns, J, h, 8)
    assert ei.value.status == _lib.SG_EINVAL


def test_reserve_then_capture(torch_dev):
    """sg_reserve sizes a fresh stream's workspace, so the first call on that
    stream can be captured into a graph directly."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, S = 48, 32
    Ns, J, h = make_batch(B, 8, 24, 11, False)
    Nt, Jt, ht = (torch.from_numpy(x).cuda() for x in (Ns, J, h))
    m0, e0 = sg.low_spectrum_batched(Nt, Jt, ht, S)  # reference on the default stream
    stream = torch.cuda.Stream()
    assert sg.sg_reserve(B, J.shape[1], S, stream) == 0
    m_out = torch.zeros((B, S), dtype=torch.int64, device="cuda")
    e_out = torch.zeros((B, S), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        st = sg.sg_low_spectrum_batched_f32(B, Nt, J.shape[1], Jt, ht, S, m_out, e_out, stream)
    assert st == 0
    for rep in range(2):
        m_out.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(m_out, m0) and torch.equal(e_out, e0), "replay %d differs" % rep
    assert sg.sg_get_error(stream) == 0


def test_graph_survives_workspace_growth(torch_dev):
    """A graph captured after sg_reserve keeps its buffers: a larger eager call
    on the same stream grows the workspace (new buffers, the old ones kept),
    and the graph still replays to the eager result; a call under capture
    that needs more than the workspace holds is refused (SG_EINVAL) instead
    of allocating."""
    import paper_1904_03621_amd as sg
    from paper_1904_03621_amd import _lib
    torch = torch_dev
    B, S, Nmax = 32, 16, 18
    Ns, J, h = make_batch(B, 8, Nmax, 13, False)
    Nt, Jt, ht = (torch.from_numpy(x).cuda() for x in (Ns, J, h))
    m0, e0 = sg.low_spectrum_batched(Nt, Jt, ht, S)
    stream = torch.cuda.Stream()
    assert sg.sg_reserve(B, Nmax, S, stream) == 0
    m_out = torch.zeros((B, S), dtype=torch.int64, device="cuda")
    e_out = torch.zeros((B, S), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        st = sg.sg_low_spectrum_batched_f32(B, Nt, Nmax, Jt, ht, S, m_out, e_out, stream)
    assert st == 0
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(m_out, m0) and torch.equal(e_out, e0)
    # a larger eager call on the graph's stream: more instances and states
    B2, S2 = 512, 64
    Ns2, J2, h2 = make_batch(B2, 8, Nmax, 14, False)
    N2t, J2t, h2t = (torch.from_numpy(x).cuda() for x in (Ns2, J2, h2))
    with torch.cuda.stream(stream):
        m2, e2 = sg.low_spectrum_batched(N2t, J2t, h2t, S2, stream=stream)
    m2d, e2d = sg.low_spectrum_batched(N2t, J2t, h2t, S2)  # default stream
    torch.cuda.synchronize()
    assert torch.equal(m2, m2d) and torch.equal(e2, e2d)
    for rep in range(2):
        m_out.fill_(-1)
        e_out.fill_(0)
        _ = torch.randn(1000, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(m_out, m0) and torch.equal(e_out, e0), "replay %d after growth" % rep
    assert sg.sg_get_error(stream) == 0
    # under capture, a call beyond the workspace is refused
    B3 = 2048
    Ns3, J3, h3 = make_batch(B3, 8, Nmax, 15, False)
    N3t, J3t, h3t = (torch.from_numpy(x).cuda() for x in (Ns3, J3, h3))
    m3 = torch.empty((B3, S), dtype=torch.int64, device="cuda")
    e3 = torch.empty((B3, S), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g3 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g3, stream=stream):
        st3 = sg.sg_low_spectrum_batched_f32(B3, N3t, Nmax, J3t, h3t, S, m3, e3, stream)
    assert st3 == _lib.SG_EINVAL, st3
    assert "capturing" in _lib.last_error()


def test_overflowing_level_is_walked_again(orc, torch_dev):
    """A strong field on the top spin puts ~55000 states of the last level
    below the threshold that the first half of the state space leaves; with
    2048 instances each has 8192 candidate slots, so that level overflows,
    is merged in part and walked again with the tighter threshold."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, N, S = 2048, 20, 64
    J0, h0 = I.random_f32_dense(N, 71, j_scale=1.0 / np.sqrt(N), h_scale=0.1)
    h0 = h0.copy()
    h0[N - 1] = 3.0
    Ns, J, h = make_batch(B, 7, 10, 12, False, Nmax=N)
    Ns[0] = N
    J[0], h[0] = J0, h0
    bm, be = run_batched(torch, Ns, J, h, S)
    info = sg.run_info()
    assert info["repeated_passes"] >= 1 and info["max_chunk_candidates"] > 8192, info
    om, oe = orc.low_spectrum(J0, h0, S)
    check_f32(N, J0, bm[0], be[0], om, oe, lambda x: orc.energy(J0, h0, x), "overflow instance")
    sm, se = run_single(torch, J0, h0, S)
    assert np.array_equal(sm, bm[0]) and np.array_equal(se, be[0])
    for b in range(1, B, 97):
        n = int(Ns[b])
        om, oe = orc.low_spectrum(J[b, :n, :n], h[b, :n], min(S, 1 << n))
        k = len(om)
        check_f32(n, J[b, :n, :n], bm[b, :k], be[b, :k], om, oe,
                  lambda x: orc.energy(J[b, :n, :n], h[b, :n], x), "instance %d" % b)


def test_full_workload_4096(orc, torch_dev):
    """The full batch: 4096 instances, N_b uniform in [16, 32], J ~ N(0,1)
    unscaled, h ~ N(0, 0.1^2), S = 64, the launch configuration the benchmark
    times.  Every instance bit for bit against the single-instance search;
    instances with N_b <= 22 (sampled) against the oracle."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    w = I.workload("batch4096")
    Ns, J, h, S = w["Ns"], w["J"], w["h"], w["S"]
    B = len(Ns)
    bm, be = run_batched(torch, Ns, J, h, S)
    # one single-instance call per instance, all on one stream
    Jb = [torch.from_numpy(np.ascontiguousarray(J[b, :Ns[b], :Ns[b]])).cuda() for b in range(B)]
    hb = [torch.from_numpy(np.ascontiguousarray(h[b, :Ns[b]])).cuda() for b in range(B)]
    sm = torch.empty((B, S), dtype=torch.int64, device="cuda")
    se = torch.empty((B, S), dtype=torch.float32, device="cuda")
    for b in range(B):
        assert sg.sg_low_spectrum_f32(int(Ns[b]), Jb[b], hb[b], S, sm[b], se[b]) == 0
    assert sg.sg_get_error() == 0
    sm = sm.cpu().numpy().astype(np.uint64)
    se = se.cpu().numpy()
    diff = [b for b in range(B) if not (np.array_equal(sm[b], bm[b]) and np.array_equal(se[b], be[b]))]
    assert not diff, "instances differing from the single search: %s" % diff[:10]
    small = [b for b in range(B) if Ns[b] <= 22][::50]
    assert len(small) >= 8
    for b in small:
        n = int(Ns[b])
        om, oe = orc.low_spectrum(J[b, :n, :n], h[b, :n], S)
        check_f32(n, J[b, :n, :n], bm[b], be[b], om, oe,
                  lambda x: orc.energy(J[b, :n, :n], h[b, :n], x), "instance %d" % b)


def test_tuner_keeps_results(torch_dev):
    """The tuner times every level geometry and keeps the fastest; the search is
    exact, so the results are the same before and after tuning."""
    import paper_1904_03621_amd as sg
    torch = torch_dev
    B, S = 96, 16
    Ns, J, h = make_batch(B, 10, 23, 13, False, Nmax=24)
    Nt, Jt, ht = (torch.from_numpy(x).cuda() for x in (Ns, J, h))
    m0, e0 = sg.low_spectrum_batched(Nt, Jt, ht, S)
    shift = sg.sg_tune_batched_f32(B, Nt, J.shape[1], Jt, ht, S)
    assert 0 <= shift <= 40
    m1, e1 = sg.low_spectrum_batched(Nt, Jt, ht, S)
    assert torch.equal(m0, m1) and torch.equal(e0, e1)


def test_maximum_S_batched(orc, torch_dev):
    """S = SG_MAX_S_BATCHED (4096) over instances of 12..16 spins."""
    B, S = 12, 4096
    Ns, J, h = make_batch(B, 12, 16, 14, True)
    bm, be = run_batched(torch_dev, Ns, J, h, S)
    for b in range(B):
        n = int(Ns[b])
        om, oe = orc.low_spectrum(J[b, :n, :n], h[b, :n], S)
        check_int(bm[b], be[b], om, oe, "batch S=4096 instance %d" % b)
