"""Parity at the full 128 x 128 workload (16384 x 16384 library, the size the
benchmark times), in the same launch configuration, on outputs the oracle
can compute one by one: sampled library columns, images of scenes supported
on those columns, and properties that hold at any size (flux, adjoint
identity)."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

FP32_REL = 1e-5
LIB_REL = 1e-6
U16 = {"bf16": 2.0**-8, "fp16": 2.0**-11}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def c2():
    return synth.config_inputs(2)


@pytest.fixture(scope="module")
def sample(c2):
    N = c2["N"]
    rng = synth.rng_for(2, synth.STREAM_SUBSAMPLE)
    C = N // 2
    special = [0, N - 1, N * N - 1, N * (N - 1), C * N + C, (C - 1) * N + C - 1, C * N + N - 1,
               (N - 1) * N + C]
    cols = np.unique(np.concatenate([rng.choice(N * N, 56, replace=False), special]))
    A = O.build_library(c2["cube"], c2["radii"], N, c2["S"], columns=cols)
    return cols, A


def _build(torch, c2, storage):
    from paper_2106_09122_amd import psflib
    return psflib.Library(torch.from_numpy(c2["cube"]).cuda(), c2["radii"], c2["N"], c2["S"],
                          storage=storage)


def _sparse_scenes(cols, ncols, B, seed):
    rng = np.random.default_rng(seed)
    Z = np.zeros((B, ncols), dtype=np.float32)
    Z[:, cols] = (rng.random((B, cols.size)) * 10.0 ** rng.uniform(-9, -7, (B, cols.size))).astype(np.float32)
    return Z


def test_c2_fp32_sampled(torch, c2, sample):
    cols, Aref = sample
    lib = _build(torch, c2, "fp32")
    got = lib.get_columns(cols).cpu().numpy().T.astype(np.float64)
    pos = Aref > 0
    assert np.all(got[~pos] == 0)
    assert np.max(np.abs(got[pos] - Aref[pos]) / Aref[pos]) <= LIB_REL
    tau = lib.column_sums().cpu().numpy()
    np.testing.assert_allclose(tau[cols], Aref.sum(axis=0), rtol=LIB_REL, atol=0)
    # single scene supported on the sampled columns
    Zs = _sparse_scenes(cols, c2["N"] ** 2, 1, 1)[0]
    ref = Aref @ Zs[cols].astype(np.float64)
    img = lib.apply(torch.from_numpy(Zs).cuda()).cpu().numpy()
    pos = ref > 0
    assert np.all(img[~pos] == 0)
    assert np.max(np.abs(img[pos] - ref[pos]) / ref[pos]) <= FP32_REL
    # the benchmark's scene: flux and adjoint identity
    Z = c2["scene"]
    S = lib.apply(torch.from_numpy(Z).cuda()).cpu().numpy().astype(np.float64)
    assert abs(S.sum() - tau @ Z.astype(np.float64)) <= 1e-5 * (tau @ Z.astype(np.float64))
    g = np.random.default_rng(2).standard_normal(c2["n"] ** 2).astype(np.float32)
    G = lib.apply_adjoint(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    lhs, rhs = S @ g.astype(np.float64), Z.astype(np.float64) @ G
    assert abs(lhs - rhs) <= 1e-5 * (np.abs(S) @ np.abs(g))
    Gref = Aref.T @ g.astype(np.float64)
    den = np.abs(Aref).T @ np.abs(g.astype(np.float64))
    assert np.all(G[cols][den == 0] == 0)
    assert np.max(np.abs(G[cols] - Gref) / np.maximum(den, 1e-300)) <= FP32_REL
    # batched: scenes supported on the sampled columns
    for B in (1, 64, 257):
        Zb = _sparse_scenes(cols, c2["N"] ** 2, B, 10 + B)
        refb = Zb[:, cols].astype(np.float64) @ Aref.T
        outb = lib.apply_batched(torch.from_numpy(Zb).cuda()).cpu().numpy()
        pos = refb > 0
        assert np.all(outb[~pos] == 0)
        assert np.max(np.abs(outb[pos] - refb[pos]) / refb[pos]) <= FP32_REL, B
    lib.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_c2_16bit_sampled(torch, c2, sample, fmt):
    cols, Aref = sample
    lib = _build(torch, c2, fmt)
    e_ref = O.pow2_exponents(O.column_max_bound(c2["cube"], c2["radii"], c2["N"], c2["S"]))
    assert np.array_equal(lib.exponents().cpu().numpy(), e_ref)
    u = U16[fmt]
    deq = lib.get_columns(cols).cpu().numpy().T.astype(np.float64)
    tol = (u * (1 + 1e-5) + LIB_REL) * Aref + 2.0**-25 * np.ldexp(1.0, e_ref[cols])[None, :]
    assert np.all(np.abs(deq - Aref) <= tol)
    # stored mantissas (dequantised values are exact float32 M 2^e) against the
    # oracle's RN(A 2^-e): equal wherever the GPU's float32 entry (within 1e-6
    # of the FP64 one) and the FP64 entry round alike, i.e. no rounding
    # boundary of the format lies within 2e-6 of the exact scaled value;
    # elsewhere one of the two neighbours of that boundary
    ec = e_ref[cols].astype(np.int64)[None, :]
    M_gpu = np.ldexp(deq, -ec)
    v = np.ldexp(Aref, -ec)
    M_ref = O.quantize_library(Aref, e_ref[cols], fmt)
    lo, hi = O.round_to_format(v * (1 - 2e-6), fmt), O.round_to_format(v * (1 + 2e-6), fmt)
    same = lo == hi
    assert np.array_equal(M_gpu[same], M_ref[same])
    assert np.all((M_gpu[~same] == lo[~same]) | (M_gpu[~same] == hi[~same]))
    assert same.mean() > 0.99
    Zs = _sparse_scenes(cols, c2["N"] ** 2, 1, 3)[0]
    ref = Aref @ Zs[cols].astype(np.float64)
    img = lib.apply(torch.from_numpy(Zs).cuda()).cpu().numpy()
    big = ref > 1e-6 * ref.max()
    assert np.max(np.abs(img - ref)[big] / ref[big]) <= u + FP32_REL
    g = np.random.default_rng(6).standard_normal(c2["n"] ** 2).astype(np.float32)
    G = lib.apply_adjoint(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    den = np.abs(Aref).T @ np.abs(g.astype(np.float64))
    assert np.all(G[cols][den == 0] == 0)
    err = np.abs(G[cols] - Aref.T @ g.astype(np.float64)) / np.maximum(den, 1e-300)
    assert np.max(err) <= u + FP32_REL
    for B in (1, 64, 300):
        Zb = _sparse_scenes(cols, c2["N"] ** 2, B, 20 + B)
        refb = Zb[:, cols].astype(np.float64) @ Aref.T
        outb = lib.apply_batched(torch.from_numpy(Zb).cuda()).cpu().numpy()
        err = np.max(np.abs(outb - refb), axis=1) / np.max(np.abs(refb), axis=1)
        assert np.max(err) <= 2 * u, (B, np.max(err))
    lib.close()


@pytest.fixture(scope="module")
def full_A(c2):
    """The whole oracle library at 128^2 (float64, 2 GiB), built in column chunks."""
    N = c2["N"]
    K = N * N
    A = np.empty((c2["n"] ** 2, K))
    for c0 in range(0, K, 2048):
        cols = np.arange(c0, min(K, c0 + 2048))
        A[:, cols] = O.build_library(c2["cube"], c2["radii"], N, c2["S"], columns=cols)
    return A


@pytest.fixture(scope="module")
def dense(c2, full_A):
    """Dense scenes over every column of the full library, with expected
    images from the whole oracle library, so every term of every accumulation
    chain is exercised (1024 scenes: a full pass of the widest 16-bit tile)."""
    Zb = np.random.default_rng(31).random((1024, c2["N"] ** 2)).astype(np.float32)
    return Zb, Zb.astype(np.float64) @ full_A.T


def _dense_single_scenes(c2):
    """The benchmark's own scene (ring + 5 planets), a dense uniform scene and a
    dense scene whose values span three decades (1e-9 to 1e-7, the ring's and
    planets' range), each over every column."""
    rng = np.random.default_rng(41)
    K = c2["N"] ** 2
    return [("bench scene", c2["scene"]),
            ("dense uniform", rng.random(K).astype(np.float32)),
            ("dense 1e-9..1e-7", (rng.random(K) * 10.0 ** rng.uniform(-9, -7, K)).astype(np.float32))]


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_c2_apply_dense(torch, c2, full_A, storage):
    """The headline single-scene product (Sec. 3, Eq. (6)) at the size and in
    the launch shape the benchmark times, compared pixel by pixel with the
    whole FP64 oracle library: every 16384-term sum runs through the blocked
    chains and split-K partials the per-pixel bound depends on.

    FP32: relative 1e-5 per pixel, exact zeros.  16-bit: every term is
    non-negative and each stored entry is within u |A_ij| of the exact one
    (u = 2^-8 BF16, 2^-11 FP16), so |dS_i| <= (u + 1e-5) S_i, plus, for FP16,
    half the subnormal spacing 2^-25 2^e_j per column for entries below the
    normal range."""
    lib = _build(torch, c2, storage)
    e = None if storage == "fp32" else lib.exponents().cpu().numpy()
    for name, Z in _dense_single_scenes(c2):
        ref = full_A @ Z.astype(np.float64)
        img = lib.apply(torch.from_numpy(Z).cuda()).cpu().numpy().astype(np.float64)
        if storage == "fp32":
            pos = ref > 0
            assert np.all(img[~pos] == 0), name
            assert np.max(np.abs(img[pos] - ref[pos]) / ref[pos]) <= FP32_REL, name
        else:
            u = U16[storage]
            sub = 2.0**-25 * float(np.ldexp(1.0, e.astype(np.int64)) @ Z.astype(np.float64)) \
                if storage == "fp16" else 0.0
            assert np.all(np.abs(img - ref) <= (u + FP32_REL) * ref + sub), name
            big = ref > 1e-6 * ref.max()
            assert np.max(np.abs(img - ref)[big] / ref[big]) <= u + FP32_REL, name
    lib.close()


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_c2_batched_dense(torch, c2, dense, storage):
    Zb, ref = dense
    lib = _build(torch, c2, storage)
    # a few scenes (mostly-padding tiles, the most K slices), then every K-split
    # shape of the GEMMs down to no split (the longest chains), an odd batch that
    # leaves the 8-wave 16-bit kernel a part-filled scene tile and a half-padding
    # staging pair, and a full pass of 1024 scenes (the 16-bit forms' 256-scene tiles)
    for B in (2, 3, 5, 8, 20, 64, 256, 301, 512, 1024):
        out = lib.apply_batched(torch.from_numpy(Zb[:B]).cuda()).cpu().numpy().astype(np.float64)
        r = ref[:B]
        if storage == "fp32":
            pos = r > 0
            assert np.all(out[~pos] == 0)
            assert np.max(np.abs(out[pos] - r[pos]) / r[pos]) <= FP32_REL, B
        else:
            # the scene is rounded to the format too: 2u per term, all terms >= 0
            u = U16[storage]
            err = np.max(np.abs(out - r), axis=1) / np.max(np.abs(r), axis=1)
            assert np.max(err) <= 2 * u, (B, np.max(err))
            big = r > 1e-3 * np.max(r, axis=1, keepdims=True)
            assert np.max(np.abs(out - r)[big] / r[big]) <= 2 * u + FP32_REL, B
    lib.close()


MODES = {
    "nearest": dict(interp="nearest"),
    "cubic": dict(rotate="cubic"),
    "flux": dict(flux="preserve"),
    "cubic_flux": dict(rotate="cubic", flux="preserve"),
}


@pytest.mark.parametrize("mode", list(MODES))
def test_c2_modes_sampled(torch, c2, sample, mode):
    """The build modes the bench times at 128^2 (nearest radial samples,
    cubic-spline rotation by orbits from staged boxes, flux-preserving columns) on the
    sampled columns and a scene supported on them.  Bounds as in the small-size
    tests of each mode: non-negative entries relative (1e-6, 2e-6 rescaled),
    cubic ones against the column bound b_j (times |s_j| when rescaled)."""
    from paper_2106_09122_amd import psflib
    kw = MODES[mode]
    cols = sample[0]
    N = c2["N"]
    A = O.build_library(c2["cube"], c2["radii"], N, c2["S"], columns=cols, **kw)
    lib = psflib.Library(torch.from_numpy(c2["cube"]).cuda(), c2["radii"], N, c2["S"], **kw)
    got = lib.get_columns(cols).cpu().numpy().T.astype(np.float64)
    cubic = kw.get("rotate") == "cubic"
    flux = kw.get("flux") == "preserve"
    Zs = _sparse_scenes(cols, N * N, 1, 71)[0]
    z = Zs[cols].astype(np.float64)
    img = lib.apply(torch.from_numpy(Zs).cuda()).cpu().numpy().astype(np.float64)
    ref = A @ z
    if not cubic:
        pos = A > 0
        assert np.all(got[~pos] == 0)
        assert np.max(np.abs(got[pos] - A[pos]) / A[pos]) <= (2e-6 if flux else LIB_REL)
        pos = ref > 0
        assert np.all(img[~pos] == 0)
        assert np.max(np.abs(img[pos] - ref[pos]) / ref[pos]) <= FP32_REL
    else:
        b = O.column_max_bound(c2["cube"], c2["radii"], N, c2["S"], rotate="cubic")[cols]
        if flux:
            A0 = O.build_library(c2["cube"], c2["radii"], N, c2["S"], columns=cols, rotate="cubic")
            tau0, t = A0.sum(axis=0), A.sum(axis=0)
            sc = np.where(tau0 != 0, t / np.where(tau0 != 0, tau0, 1.0), 1.0)
            eb = 2e-6 * np.abs(sc) * b
        else:
            eb = 1e-6 * b
        assert np.all(np.abs(got - A) <= eb[None, :] + 1e-300)
        assert np.all(np.abs(img - ref) <= FP32_REL * (np.abs(A) @ z) + eb @ z + 1e-300)
    if flux:
        tau = lib.column_sums().cpu().numpy()[cols]
        t = A.sum(axis=0)
        live = t != 0
        assert np.all(tau[~live] == 0)
        assert np.max(np.abs(tau[live] - t[live]) / np.abs(t[live])) <= 1e-6
    lib.close()


def test_paper_shape_sampled(torch):
    """The paper's own shape (128^2 PSFs at 0.2 lambda/D with the non-uniform
    IPAC offsets, a 256^2 scene at 3.529 mas: n != N, s != S, a 16384 x 65536
    library) on 64 seeded columns and a scene supported on them."""
    from paper_2106_09122_amd import psflib
    d = synth.config_inputs(6)
    N = d["N"]
    rng = synth.rng_for(6, synth.STREAM_SUBSAMPLE)
    cols = np.sort(rng.choice(N * N, 64, replace=False))
    Aref = O.build_library(d["cube"], d["radii"], N, d["S"], columns=cols)
    lib = psflib.Library(torch.from_numpy(d["cube"]).cuda(), d["radii"], N, d["S"])
    got = lib.get_columns(cols).cpu().numpy().T.astype(np.float64)
    pos = Aref > 0
    assert np.all(got[~pos] == 0)
    assert np.max(np.abs(got[pos] - Aref[pos]) / Aref[pos]) <= LIB_REL
    Zs = _sparse_scenes(cols, N * N, 1, 61)[0]
    ref = Aref @ Zs[cols].astype(np.float64)
    img = lib.apply(torch.from_numpy(Zs).cuda()).cpu().numpy()
    pos = ref > 0
    assert np.all(img[~pos] == 0)
    assert np.max(np.abs(img[pos] - ref[pos]) / ref[pos]) <= FP32_REL
    # a few scenes at once (more columns than image rows)
    Zb = _sparse_scenes(cols, N * N, 6, 62)
    refb = Zb[:, cols].astype(np.float64) @ Aref.T
    out = lib.apply_batched(torch.from_numpy(Zb).cuda()).cpu().numpy()
    pos = refb > 0
    assert np.all(out[~pos] == 0)
    assert np.max(np.abs(out[pos] - refb[pos]) / refb[pos]) <= FP32_REL
    lib.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_paper_shape_16bit_sampled(torch, fmt):
    """The paper's shape (n = 128 != N = 256, non-uniform offsets, 16384 x 65536)
    in the 16-bit forms: exponents bitwise, sampled dequantised columns, and a
    single and a batched product of scenes supported on those columns."""
    from paper_2106_09122_amd import psflib
    d = synth.config_inputs(6)
    N = d["N"]
    rng = synth.rng_for(6, synth.STREAM_SUBSAMPLE)
    cols = np.sort(rng.choice(N * N, 64, replace=False))
    Aref = O.build_library(d["cube"], d["radii"], N, d["S"], columns=cols)
    lib = psflib.Library(torch.from_numpy(d["cube"]).cuda(), d["radii"], N, d["S"], storage=fmt)
    e_ref = O.pow2_exponents(O.column_max_bound(d["cube"], d["radii"], N, d["S"]))
    assert np.array_equal(lib.exponents().cpu().numpy(), e_ref)
    u = U16[fmt]
    deq = lib.get_columns(cols).cpu().numpy().T.astype(np.float64)
    tol = (u * (1 + 1e-5) + LIB_REL) * Aref + 2.0**-25 * np.ldexp(1.0, e_ref[cols])[None, :]
    assert np.all(np.abs(deq - Aref) <= tol)
    Zs = _sparse_scenes(cols, N * N, 1, 63)[0]
    ref = Aref @ Zs[cols].astype(np.float64)
    img = lib.apply(torch.from_numpy(Zs).cuda()).cpu().numpy()
    big = ref > 1e-6 * ref.max()
    assert np.max(np.abs(img - ref)[big] / ref[big]) <= u + FP32_REL
    Zb = _sparse_scenes(cols, N * N, 6, 64)
    refb = Zb[:, cols].astype(np.float64) @ Aref.T
    outb = lib.apply_batched(torch.from_numpy(Zb).cuda()).cpu().numpy()
    err = np.max(np.abs(outb - refb), axis=1) / np.max(np.abs(refb), axis=1)
    assert np.max(err) <= 2 * u, np.max(err)
    lib.close()


@pytest.fixture(scope="module")
def c4_data(c2, full_A):
    """Fit data at 128^2: the oracle's image of the true disk plus seeded
    Poisson and Gaussian noise (no expected value depends on the HIP path)."""
    counts, K, var = synth.noisy_counts(full_A @ O.render_disk(c2["N"], c2["S"], RMAX, synth.DISK_TRUE),
                                        2e4, synth.rng_for(4, synth.STREAM_NOISE))
    return counts, K, var


RMAX = 8.0


def test_c2_fit_step_gradient(torch, c2, full_A, c4_data):
    """The fit step the bench times at 128^2 (render -> A Z -> chi-square ->
    A^T -> renderer gradient), component by component, against (i) the FP64
    oracle chain on the whole library, under each component's own error scale
    (the chain evaluated on |r| + K S, |A| and |dZ/dtheta_k|), and (ii) FP64
    central differences of the oracle loss in each parameter."""
    import chi2_chain as C
    from paper_2106_09122_amd import fit
    N, S = c2["N"], c2["S"]
    counts, K, var = c4_data
    lib = _build(torch, c2, "fp32")
    th0 = synth.DISK_START
    th = torch.tensor(th0, dtype=torch.float64, device="cuda")
    L, g = fit.loss_and_grad(lib, th, torch.from_numpy(counts).cuda(), torch.from_numpy(var).cuda(),
                             K, RMAX)
    g = g.cpu().numpy()
    Lref, gref = C.loss_and_grad(full_A, N, S, RMAX, th0, counts, var, K)
    scale, scale_r = C.gradient_scales(full_A, N, S, RMAX, th0, counts, var, K)
    assert abs(float(L) - Lref) <= 1e-4 * Lref
    # per component: within the propagated float32 error bound, and within
    # 2e-3 of the chain evaluated on |r| (a looser, simpler scale)
    assert np.all(np.abs(g - gref) <= 2e-5 * scale), (g, gref, scale)
    assert np.all(np.abs(g - gref) <= 2e-3 * scale_r), (g, gref, scale_r)
    fd = C.central_differences(full_A, N, S, RMAX, th0, counts, var, K)
    assert np.all(np.abs(gref - fd) <= 1e-8 * np.abs(fd)), (gref, fd)  # the oracle itself
    assert np.all(np.abs(g - fd) <= 2e-5 * scale + 1e-6 * np.abs(fd)), (g, fd)
    lib.close()


def test_c2_fit_64_steps(torch, c2, c4_data):
    """The retrieval at the configured size: 64 Adam steps at 128^2 through the
    operator and its adjoint reduce the chi-square and move the disk's
    geometry (inclination, radius, width) toward the truth (the paper's
    planned parameter retrieval, Sec. 5)."""
    from paper_2106_09122_amd import fit
    counts, K, var = c4_data
    lib = _build(torch, c2, "fp32")
    theta, losses = fit.fit_disk(lib, torch.from_numpy(counts).cuda(), torch.from_numpy(var).cuda(),
                                 K, synth.DISK_START, RMAX, steps=64)
    assert len(losses) == 64
    assert losses[-1] < 0.05 * losses[0], (losses[0], losses[-1])
    t = theta.cpu().numpy()
    tt, t0 = np.array(synth.DISK_TRUE), np.array(synth.DISK_START)
    for k in (0, 1, 2):
        assert abs(t[k] - tt[k]) < abs(t0[k] - tt[k]), (k, t, tt, t0)
    lib.close()
