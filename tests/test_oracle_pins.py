"""Pins for the FP64 oracle: values the paper prints, library routines the
method reduces to in special cases, closed forms, invariants and brute force.

Each test is chosen so that a plausible mistake in the oracle (a dropped
half-pixel shift, swapped axes, a wrong rotation sense or centre, an
off-by-one bracket, a transposed product) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.interpolate import RegularGridInterpolator

import oracle as O
from tests.conftest import golden

G = golden("paper_values.txt")
MAS_PER_RAD = 180.0 / math.pi * 3600e3


# ----------------------------------------------------------- geometry ------
def test_constants_consistent_with_paper():
    """Eq. (1): 0.2 lambda/D = 10.038 mas and 256 x 3.529 mas / 2 = 9 lambda/D."""
    lod_mas = G["wavelength_nm"] * 1e-9 / G["diameter_m"] * MAS_PER_RAD
    assert abs(G["psf_pixscale_lod"] * lod_mas - G["psf_pixscale_mas"]) < 5e-4
    half_extent = G["scene_npx"] / 2 * G["scene_pixscale_mas"] / lod_mas
    assert abs(half_extent - G["scene_extent_lod"]) < 1e-3


def test_field_point_printed_in_paper_is_a_scene_pixel():
    """Figs. 3 and 8 quote a field point of 286.838 mas at 66.431 deg on the
    256 px, 3.529 mas scene.  With the half-pixel-shifted meshgrid of Eqs.
    (2)-(3), x along columns and y along rows, exactly one scene pixel has
    that offset to the printed precision (row 202, col 160); without the
    half-pixel shift, or with the axes swapped, none does."""
    N = int(G["scene_npx"])
    S = G["scene_pixscale_mas"]
    x, y, r, ct, st = O.scene_geometry(N, S)
    theta = np.degrees(np.arctan2(st, ct))
    hit = np.nonzero((np.abs(r - G["field_point_r_mas"]) < 5e-4)
                     & (np.abs(theta - G["field_point_theta_deg"]) < 5e-4))[0]
    assert hit.tolist() == [202 * N + 160]
    # the unshifted grid gives no such pixel
    t = (np.arange(N) - N / 2) * S
    xu, yu = np.meshgrid(t, t)
    ru = np.hypot(xu, yu)
    tu = np.degrees(np.arctan2(yu, xu))
    assert not np.any((np.abs(ru - G["field_point_r_mas"]) < 5e-4)
                      & (np.abs(tu - G["field_point_theta_deg"]) < 5e-4))


def test_geometry_layout_and_polar_form():
    N, S = 7, 0.5
    x, y, r, ct, st = O.scene_geometry(N, S)
    X = x.reshape(N, N)
    Y = y.reshape(N, N)
    assert np.all(np.diff(X, axis=1) == S) and np.all(np.diff(X, axis=0) == 0)
    assert np.all(np.diff(Y, axis=0) == S) and np.all(np.diff(Y, axis=1) == 0)
    assert X[0, 0] == -1.5 and Y[0, 0] == -1.5 and X[3, 3] == 0 and Y[3, 3] == 0
    c = N // 2 * N + N // 2
    assert r[c] == 0 and ct[c] == 1 and st[c] == 0  # atan2(0, 0) = 0
    nz = r > 0
    np.testing.assert_allclose(ct[nz], np.cos(np.arctan2(y[nz], x[nz])), atol=1e-15)
    np.testing.assert_allclose(st[nz], np.sin(np.arctan2(y[nz], x[nz])), atol=1e-15)
    # even N has no pixel on the optical axis and is symmetric
    _, _, r8, _, _ = O.scene_geometry(8, 1.0)
    assert r8.min() > 0 and np.allclose(np.sort(r8), np.sort(r8[::-1]))


# --------------------------------------------------------------- shape -----
def test_library_shape_matches_table2_file_sizes():
    """Table 2: 8 GB for 128 px PSFs and 32 GB for 256 px PSFs on a 256 px
    scene: A is n^2 x N^2 float64 (Sec. 3: n^2 rows, N^2 columns)."""
    assert (G["psf_npx"] ** 2) * (G["scene_npx"] ** 2) * 8 == G["ipac_library_gb"] * 2**30
    assert (G["proper_npx"] ** 2) * (G["scene_npx"] ** 2) * 8 == G["proper_library_gb"] * 2**30
    assert round(G["proper_max_offset_lod"] / G["proper_offset_step_lod"]) + 1 == G["proper_n_psf"]
    rng = np.random.default_rng(0)
    cube = rng.random((3, 5, 5))
    A = O.build_library(cube, [0.0, 1.0, 2.0], N=4, S=0.7)
    assert A.shape == (25, 16)


# -------------------------------------------------------------- radial -----
@pytest.mark.parametrize("method", ["linear", "nearest"])
def test_radial_matches_regular_grid_interpolator(method):
    """At integer pixel nodes the paper's RegularGridInterpolator over
    (offset, y, x) reduces to interpolation in offset alone."""
    rng = np.random.default_rng(1)
    n, K = 6, 9
    radii = np.cumsum(rng.uniform(0.1, 1.0, K))
    cube = rng.random((K, n, n))
    f = RegularGridInterpolator((radii, np.arange(n), np.arange(n)), cube, method=method)
    aa, bb = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for r in rng.uniform(radii[0], radii[-1], 40):
        k, w, zero = O.radial_bracket(r, radii, method)
        assert not zero
        Q = O.interpolate_radial(cube, k, w)
        pts = np.stack([np.full(n * n, r), aa.ravel(), bb.ravel()], axis=1)
        np.testing.assert_allclose(Q.ravel(), f(pts), rtol=1e-13, atol=1e-15)


def test_radial_samples_ties_and_range():
    radii = np.array([0.0, 0.5, 2.0, 3.0])
    assert O.radial_bracket(0.5, radii) == (1, 0.0, False)     # exact sample: w = 0
    assert O.radial_bracket(2.0, radii) == (2, 0.0, False)
    assert O.radial_bracket(3.0, radii) == (2, 1.0, False)     # last sample
    assert O.radial_bracket(-1.0, radii) == (0, 0.0, False)    # below: first PSF
    assert O.radial_bracket(9.0, radii) == (2, 1.0, False)     # clamp
    assert O.radial_bracket(9.0, radii, oob="zero")[2] is True
    assert O.radial_bracket(3.0, radii, oob="zero") == (2, 1.0, False)
    assert O.radial_bracket(1.25, radii, "nearest") == (1, 0.0, False)  # tie -> lower
    assert O.radial_bracket(1.26, radii, "nearest") == (1, 1.0, False)
    k, w, _ = O.radial_bracket(1.25, radii)
    assert k == 1 and w == 0.5
    assert O.radial_bracket(5.0, np.array([1.0])) == (0, 0.0, False)


# ------------------------------------------------------------ rotation -----
@pytest.mark.parametrize("n", [8, 9, 16])
@pytest.mark.parametrize("deg", [30.0, 66.431, -110.0, 200.0])
def test_rotation_matches_scipy_ndimage(n, deg):
    """Bilinear rotation about the array centre, frame kept, zero padding:
    scipy.ndimage.rotate(Q, -theta, reshape=False, order=1,
    mode='grid-constant') (scipy's positive angle turns +x towards -row)."""
    rng = np.random.default_rng(n)
    Q = rng.random((n, n))
    th = math.radians(deg)
    mine = O.rotate_bilinear(Q, math.cos(th), math.sin(th))
    ref = ndimage.rotate(Q, -deg, reshape=False, order=1, mode="grid-constant", cval=0.0)
    np.testing.assert_allclose(mine, ref, atol=1e-12, rtol=0)


@pytest.mark.parametrize("n", [6, 7])
def test_rotation_quarter_turns_are_exact(n):
    rng = np.random.default_rng(5)
    Q = rng.random((n, n))
    assert np.array_equal(O.rotate_bilinear(Q, 1.0, 0.0), Q)
    assert np.array_equal(O.rotate_bilinear(Q, 0.0, 1.0), np.rot90(Q, -1))
    assert np.array_equal(O.rotate_bilinear(Q, -1.0, 0.0), np.rot90(Q, 2))
    assert np.array_equal(O.rotate_bilinear(Q, 0.0, -1.0), np.rot90(Q, 1))


# ------------------------------------------------ cubic-spline rotation ----
def test_spline_prefilter_matches_scipy():
    """The cubic B-spline interpolation filter (mirror extension) equals
    scipy.ndimage.spline_filter1d(order=3, mode='mirror')."""
    rng = np.random.default_rng(40)
    for N in (2, 3, 7, 40, 152):
        s = rng.standard_normal(N)
        ref = ndimage.spline_filter1d(s, order=3, mode="mirror")
        np.testing.assert_allclose(O.spline_prefilter_1d(s), ref, atol=1e-13 * np.abs(ref).max(), rtol=0)


@pytest.mark.parametrize("n", [8, 9, 20])
@pytest.mark.parametrize("deg", [30.0, 66.431, -110.0, 200.0])
def test_cubic_rotation_matches_scipy_ndimage(n, deg):
    """Cubic-spline rotation of the zero-extended PSF:
    scipy.ndimage.rotate(Q, -theta, reshape=False, order=3,
    mode='grid-constant') (which pads by 12 and filters with mirror
    boundaries, the oracle's definition)."""
    rng = np.random.default_rng(100 + n)
    Q = rng.random((n, n))
    th = math.radians(deg)
    mine = O.rotate_cubic(Q, math.cos(th), math.sin(th))
    ref = ndimage.rotate(Q, -deg, reshape=False, order=3, mode="grid-constant", cval=0.0)
    np.testing.assert_allclose(mine, ref, atol=1e-12, rtol=0)


@pytest.mark.parametrize("n", [6, 7])
def test_cubic_rotation_interpolates_nodes(n):
    """A spline interpolant passes through its samples: no turn and the
    quarter turns map nodes to nodes and return the samples (to rounding)."""
    rng = np.random.default_rng(6)
    Q = rng.random((n, n))
    np.testing.assert_allclose(O.rotate_cubic(Q, 1.0, 0.0), Q, atol=1e-13, rtol=0)
    np.testing.assert_allclose(O.rotate_cubic(Q, 0.0, 1.0), np.rot90(Q, -1), atol=1e-13, rtol=0)
    np.testing.assert_allclose(O.rotate_cubic(Q, -1.0, 0.0), np.rot90(Q, 2), atol=1e-13, rtol=0)


def test_cubic_rotation_is_fourth_order():
    """Rotating samples of a smooth Gaussian with the cubic spline differs
    from samples of the rotated Gaussian by O(h^4): halving the pixel pitch
    cuts the error about 16-fold (bilinear: about 4-fold)."""
    sig, x0, half, deg = 0.6, 1.2, 4.0, 37.0
    th = math.radians(deg)
    errs_c, errs_b = [], []
    for h in (0.2, 0.1):
        n = int(round(2 * half / h)) + 1
        c = (n - 1) / 2.0
        a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        X, Y = (b - c) * h, (a - c) * h
        Q = np.exp(-((X - x0) ** 2 + Y**2) / (2 * sig**2))
        exact = np.exp(-((X - x0 * math.cos(th)) ** 2 + (Y - x0 * math.sin(th)) ** 2) / (2 * sig**2))
        errs_c.append(np.abs(O.rotate_cubic(Q, math.cos(th), math.sin(th)) - exact).max())
        errs_b.append(np.abs(O.rotate_bilinear(Q, math.cos(th), math.sin(th)) - exact).max())
    assert 10.0 < errs_c[0] / errs_c[1] < 24.0, errs_c
    assert 3.0 < errs_b[0] / errs_b[1] < 5.0, errs_b
    assert errs_c[1] < 0.05 * errs_b[1]


def test_cubic_column_bound():
    """max_i |A_ij| never exceeds (1-w) max|C_k| + w max|C_{k+1}| (spline
    coefficients of the samples), and cubic columns of on-axis field points at
    sampled offsets are the samples themselves."""
    rng = np.random.default_rng(13)
    cube = rng.random((5, 11, 11)) ** 3
    radii = np.linspace(0.0, 2.0, 5)
    bound = O.column_max_bound(cube, radii, 9, 0.5, rotate="cubic")
    A = O.build_library(cube, radii, 9, 0.5, rotate="cubic")
    assert np.all(np.abs(A).max(axis=0) <= bound * (1 + 1e-14))
    x, y, r, _, _ = O.scene_geometry(9, 0.5)
    for j in np.nonzero((np.abs(y) < 1e-12) & (x >= 0) & (x <= 2.0))[0]:
        k = int(round(x[j] / 0.5))
        np.testing.assert_allclose(A[:, j], cube[k].ravel(), atol=1e-13, rtol=0)


# ------------------------------------------------ flux-preserving rescale ----
def test_flux_preserving_columns():
    """flux='preserve': quarter-turn field points (bilinear rotation there is a
    permutation of pixels, no flux lost) are unchanged; elsewhere the column is
    scipy's rotation of the interpolated PSF scaled to the PSF's own total,
    which leaves the frame partly for field points far off-axis."""
    n, N, S = 15, 9, 0.7
    rng = np.random.default_rng(31)
    cube = rng.random((4, n, n)) ** 2
    radii = np.array([0.0, 1.0, 2.5, 4.0])
    x, y, r, ct, st = O.scene_geometry(N, S)
    A0 = O.build_library(cube, radii, N, S)
    A1 = O.build_library(cube, radii, N, S, flux="preserve")
    axes = np.nonzero((np.abs(x) < 1e-12) | (np.abs(y) < 1e-12))[0]
    np.testing.assert_allclose(A1[:, axes], A0[:, axes], rtol=1e-13, atol=0)
    for j in (0, 10, 23, 40, 80):
        k, w, _ = O.radial_bracket(r[j], radii)
        Q = (1 - w) * cube[k] + w * cube[k + 1]
        deg = math.degrees(math.atan2(y[j], x[j]))
        rot = ndimage.rotate(Q, -deg, reshape=False, order=1, mode="grid-constant", cval=0.0)
        ref = (rot * (Q.sum() / rot.sum())).ravel()
        np.testing.assert_allclose(A1[:, j], ref, rtol=1e-10, atol=1e-13)
    lost = A0.sum(axis=0) < 0.999 * A1.sum(axis=0)
    assert lost.any()  # some field points do lose flux to the frame edge


def _gauss_cube(n, radii_px, sigma):
    c = (n - 1) / 2.0
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([np.exp(-((b - c - rk) ** 2 + (a - c) ** 2) / (2 * sigma**2)) for rk in radii_px])


def test_core_lands_on_field_point():
    """Pins the rotation sense: the centroid of each column is the field
    point (in image pixels, s = S), with y along increasing row index."""
    n = N = 33
    S = 1.0
    radii = np.arange(0.0, 13.0)  # in pixels
    cube = _gauss_cube(n, radii, 1.3)
    x, y, r, _, _ = O.scene_geometry(N, S)
    c = (n - 1) / 2.0
    aa, bb = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rng = np.random.default_rng(3)
    for j in rng.choice(np.nonzero((r > 2) & (r < 10))[0], 25, replace=False):
        col = O.build_library(cube, radii, N, S, columns=[j])[:, 0].reshape(n, n)
        cx = (col * bb).sum() / col.sum() - c
        cy = (col * aa).sum() / col.sum() - c
        assert abs(cx - x[j]) < 0.06 and abs(cy - y[j]) < 0.06, (j, cx, cy, x[j], y[j])


# ------------------------------------------------------- method-level ------
def test_point_source_on_axis_reproduces_sample_exactly():
    """Odd N, S = 0.5, offsets on the same 0.5 lattice: a unit source on +x
    at r = rho_k images to P_k exactly; on +y, -x and -y to its exact
    quarter-turn rotations."""
    N, S = 33, 0.5
    radii = np.arange(17) * 0.5
    rng = np.random.default_rng(11)
    n = 32
    cube = rng.random((17, n, n)).astype(np.float32)
    C = N // 2
    for m in range(0, 17):
        for (p, q, rot) in [(C, C + m, 0), (C + m, C, -1), (C, C - m, 2), (C - m, C, 1)]:
            if m == 0 and rot != 0:
                continue
            j = p * N + q
            col = O.build_library(cube, radii, N, S, columns=[j])[:, 0].reshape(n, n)
            assert np.array_equal(col, np.rot90(cube[m].astype(np.float64), rot)), (m, rot)


def _brute_column(cube, radii, N, S, j, method="linear"):
    """Library column by a different route: scipy's RegularGridInterpolator
    for the offset, atan2/cos/sin for the angle, scipy.ndimage.map_coordinates
    for the bilinear zero-padded sample."""
    K, n, _ = cube.shape
    p, q = divmod(j, N)
    x = (q - (N - 1) / 2) * S
    y = (p - (N - 1) / 2) * S
    r = math.hypot(x, y)
    th = math.atan2(y, x)
    f = RegularGridInterpolator((radii, np.arange(n), np.arange(n)), cube.astype(np.float64),
                                method=method)
    aa, bb = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rr = min(max(r, radii[0]), radii[-1])
    Q = f(np.stack([np.full(n * n, rr), aa.ravel(), bb.ravel()], 1)).reshape(n, n)
    c = (n - 1) / 2
    ux, uy = bb - c, aa - c
    cols = c + math.cos(th) * ux + math.sin(th) * uy
    rows = c - math.sin(th) * ux + math.cos(th) * uy
    return ndimage.map_coordinates(Q, [rows.ravel(), cols.ravel()], order=1,
                                   mode="grid-constant", cval=0.0)


@pytest.mark.parametrize("n,N,S", [(8, 11, 0.37), (9, 6, 0.5), (10, 10, 0.25)])
def test_library_matches_library_routines_brute_force(n, N, S):
    rng = np.random.default_rng(n * 100 + N)
    K = 7
    radii = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 0.6, K - 1))])
    cube = rng.random((K, n, n)).astype(np.float32)
    A = O.build_library(cube, radii, N, S)
    for j in range(N * N):
        np.testing.assert_allclose(A[:, j], _brute_column(cube, radii, N, S, j), atol=1e-12)


# ---------------------------------------------------- products, flux -------
def _small_problem(seed=0, n=9, N=7, K=5):
    rng = np.random.default_rng(seed)
    radii = np.linspace(0.0, 3.0, K)
    cube = rng.random((K, n, n)).astype(np.float32)
    return cube, radii, O.build_library(cube, radii, N, 0.6), rng


def test_apply_matches_python_loops_and_for_loop_form():
    """Eq. (6) by explicit Python sums over rows (math.fsum), and the
    paper's for-loop form (Sec. 3): S = sum_j Z_j I_j."""
    cube, radii, A, rng = _small_problem()
    Z = rng.random(A.shape[1])
    S = O.apply(A, Z)
    rows = [math.fsum(A[i, j] * Z[j] for j in range(A.shape[1])) for i in range(A.shape[0])]
    np.testing.assert_allclose(S, rows, rtol=1e-14)
    loop = np.zeros(A.shape[0])
    for j in range(A.shape[1]):
        loop += Z[j] * A[:, j]
    np.testing.assert_allclose(S, loop, rtol=1e-13)


def test_linearity_flux_adjoint_batched():
    cube, radii, A, rng = _small_problem(1)
    Z1, Z2 = rng.random(A.shape[1]), rng.random(A.shape[1])
    np.testing.assert_allclose(O.apply(A, 2.5 * Z1 - 0.75 * Z2),
                               2.5 * O.apply(A, Z1) - 0.75 * O.apply(A, Z2), rtol=1e-12, atol=1e-13)
    tau = O.column_sums(A)
    assert abs(O.apply(A, Z1).sum() - tau @ Z1) < 1e-12 * tau @ Z1
    g = rng.standard_normal(A.shape[0])
    assert abs(O.apply(A, Z1) @ g - Z1 @ O.apply_adjoint(A, g)) < 1e-12 * np.abs(A).sum()
    Zb = rng.random((4, A.shape[1]))
    out = O.apply_batched(A, Zb)
    for b in range(4):
        np.testing.assert_allclose(out[b], O.apply(A, Zb[b]), rtol=1e-14)


def test_oob_modes():
    n, N, S = 8, 9, 1.0
    radii = np.array([0.0, 1.0, 2.0])
    rng = np.random.default_rng(7)
    cube = rng.random((3, n, n))
    _, _, r, _, _ = O.scene_geometry(N, S)
    A_c = O.build_library(cube, radii, N, S, oob="clamp")
    A_z = O.build_library(cube, radii, N, S, oob="zero")
    out = r > 2.0
    assert np.all(A_z[:, out] == 0)
    assert np.array_equal(A_c[:, ~out], A_z[:, ~out])
    # clamped columns use the last PSF; on the +x axis that is P_{K-1} itself
    j = 4 * N + 8  # row C=4, col 8 -> x = 4 > rho_max, theta = 0
    assert np.array_equal(A_c[:, j], cube[2].ravel())


def test_nearest_columns_are_rotated_samples():
    cube, radii, _, rng = _small_problem(2)
    N, S = 7, 0.6
    An = O.build_library(cube, radii, N, S, interp="nearest")
    _, _, r, ct, st = O.scene_geometry(N, S)
    for j in range(N * N):
        cands = [O.rotate_bilinear(cube[k].astype(np.float64), ct[j], st[j]).ravel()
                 for k in range(cube.shape[0])]
        kbest = int(np.argmin(np.abs(radii - min(r[j], radii[-1]))))
        assert np.array_equal(An[:, j], cands[kbest])


# ------------------------------------------------- convolution limit -------
def _gauss(dx, dy, sig):
    return np.exp(-(dx * dx + dy * dy) / (2 * sig * sig))


def _conv_case(n, h, sig, dr):
    """Isoplanatic PSF: the same Gaussian (sigma sig, physical units)
    shifted to each sampled offset; n = N, s = S = h."""
    radii = np.arange(0.0, 3.0 + 1e-9, dr)
    c = (n - 1) / 2.0
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    cube = np.stack([_gauss((b - c) * h - rk, (a - c) * h, sig) for rk in radii])
    return radii, cube


def test_convolution_limit_exact_on_axes():
    n, h, sig = 17, 0.5, 0.6
    radii, cube = _conv_case(n, h, sig, h)
    N = n
    C = N // 2
    x, y, r, _, _ = O.scene_geometry(N, h)
    c = (n - 1) / 2.0
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ux, uy = (b - c) * h, (a - c) * h
    for m in range(0, 7):
        for (p, q) in [(C, C + m), (C + m, C), (C, C - m), (C - m, C)]:
            j = p * N + q
            col = O.build_library(cube, radii, N, h, columns=[j])[:, 0]
            brute = _gauss(ux - x[j], uy - y[j], sig).ravel()
            np.testing.assert_allclose(col, brute, rtol=1e-14, atol=1e-300)


def _conv_error(n, h, sig, rsrc):
    radii, cube = _conv_case(n, h, sig, h)
    N = n
    x, y, r, _, _ = O.scene_geometry(N, h)
    c = (n - 1) / 2.0
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ux, uy = ((b - c) * h).ravel(), ((a - c) * h).ravel()
    sel = np.nonzero((r > 0.3) & (r < rsrc))[0]
    A = O.build_library(cube, radii, N, h, columns=sel)
    err = 0.0
    for t, j in enumerate(sel):
        brute = _gauss(ux - x[j], uy - y[j], sig)
        err = max(err, np.abs(A[:, t] - brute).max())
    return err


def test_convolution_limit_error_bound_and_order():
    """Off the sampled points, the column differs from the shifted Gaussian
    by at most the closed-form linear-interpolation bound in offset,
    (dr^2/8) max|G''|, plus the bilinear bound (h^2/8)(max|G_xx|+max|G_yy|)
    (max|G''| = 1/sigma^2), plus the zero-padding tail; halving h (with
    dr = h, sigma fixed) cuts the error about four-fold."""
    sig, rsrc, half = 0.5, 1.5, 4.0
    errs = []
    for h in (0.25, 0.125):
        n = int(round(2 * half / h)) + 1
        e = _conv_error(n, h, sig, rsrc)
        bound = (h * h / 8) / sig**2 + (h * h / 8) * 2 / sig**2
        edge = half - rsrc - h  # distance from any sample core used to the frame edge
        tail = math.exp(-edge * edge / (2 * sig * sig))
        assert e <= bound + tail, (h, e, bound, tail)
        errs.append(e)
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


# --------------------------------------------------------- 16-bit forms ----
def test_round_to_format_fp16_matches_numpy():
    rng = np.random.default_rng(9)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-9, 5, 2000),
                        [0.0, 65504.0, 65519.99, 2.0**-24, 3 * 2.0**-26, 2.0**-14 * 1.5]])
    np.testing.assert_array_equal(O.round_to_format(v, "fp16"),
                                  v.astype(np.float16).astype(np.float64))


def test_round_to_format_bf16_matches_torch_on_float32_values():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(10)
    v = (rng.standard_normal(4000) * 10.0 ** rng.integers(-30, 30, 4000)).astype(np.float32)
    v = np.concatenate([v, np.float32([1 + 2**-8, 1 + 3 * 2**-8, 2.0**-130, 0.0])])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.round_to_format(v.astype(np.float64), "bf16"), ref)


def test_scale_exponent_and_bound():
    for m in [1e-30, 3e-10, 0.5, 1.0, 2.0**-20, 0.7647, 12345.6]:
        e = O.scale_exponent(m)
        assert 2**14 <= m * 2.0**-e < 2**15
    # a zero column: any finite scene value scaled by its exponent is exactly 0
    # (float32 and float64), and the column's dequantised values stay 0
    ez = O.scale_exponent(0.0)
    assert ez == O.ZERO_COLUMN_EXPONENT
    big = np.array([np.finfo(np.float32).max, 1.0, 1e-30], dtype=np.float32)
    assert np.all(np.ldexp(big, np.int32(ez)) == 0)
    assert np.all(np.ldexp(big.astype(np.float64), ez) == 0)
    assert np.all(O.quantize_library(np.zeros((5, 1)), np.array([ez]), "fp16") == 0)
    rng = np.random.default_rng(12)
    cube = rng.random((6, 12, 12)) ** 4
    radii = np.linspace(0, 2.5, 6)
    bound = O.column_max_bound(cube, radii, 9, 0.4)
    A = O.build_library(cube, radii, 9, 0.4)
    assert np.all(A.max(axis=0) <= bound * (1 + 1e-15))


def test_quantize_library_pins():
    """Mantissas M_ij = RN(A_ij 2^-e_j): pinned to the formats' own conversions
    (numpy float16, torch bfloat16), to a worked value, and to the range the
    exponent rule promises, on columns whose scales span 14 decades."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    ncol = 24
    # float32 entries (as the GPU rounds them), column scales 1e-12 .. 1e2
    A = (rng.random((300, ncol)) ** 3 * 10.0 ** rng.uniform(-12, 2, ncol)).astype(np.float32)
    A[rng.random(A.shape) < 0.05] = 0.0
    A[:, 5] = 0.0  # an identically zero column
    A = A.astype(np.float64)
    b = A.max(axis=0)
    e = O.pow2_exponents(b)
    live = b > 0
    assert e[5] == O.ZERO_COLUMN_EXPONENT
    # worked value: 3 = 0.75 * 2^2, so e = 2 - 15 = -13 and M = 3 * 2^13 = 24576
    # (an exponent of the wrong sign would give 3 * 2^-13, far below the range)
    assert O.scale_exponent(3.0) == -13
    for fmt in ("fp16", "bf16"):
        assert O.quantize_library(np.array([[3.0]]), np.array([-13]), fmt)[0, 0] == 24576.0
    scaled = np.ldexp(A, -e.astype(np.int64)[None, :])
    for fmt, u in (("fp16", 2.0**-11), ("bf16", 2.0**-8)):
        Mq = O.quantize_library(A, e, fmt)
        # the formats' own round-to-nearest-even conversions
        if fmt == "fp16":
            ref = scaled.astype(np.float16).astype(np.float64)
        else:
            ref = torch.from_numpy(scaled.astype(np.float32)).to(torch.bfloat16).double().numpy()
        np.testing.assert_array_equal(Mq, ref)
        # the largest mantissa of every live column lands in [2^14, 2^15]
        top = np.abs(Mq[:, live]).max(axis=0)
        assert np.all(top >= 2**14) and np.all(top <= 2**15), top
        # M 2^e reproduces A to the format's unit (FP16: plus half its
        # subnormal spacing 2^-25 for entries below its normal range)
        rec = np.ldexp(Mq, e.astype(np.int64)[None, :])
        sub = 2.0**-25 * np.ldexp(1.0, e.astype(np.int64))[None, :] if fmt == "fp16" else 0.0
        assert np.all(np.abs(rec - A) <= u * np.abs(A) + sub)
        assert np.all(Mq[:, 5] == 0) and np.all(Mq[A == 0] == 0)
        # a sign error in the exponent leaves the range: scaling by 2^+e
        wrong = O.round_to_format(np.ldexp(A, e.astype(np.int64)[None, :]), fmt)
        assert not np.all(np.abs(wrong[:, live]).max(axis=0) >= 2**14)


# ------------------------------------------------------ fitting model ------
THETA = (math.radians(55.0), 5.0, 1.2, -1.4, 3e-8)


def test_disk_gradient_matches_central_differences():
    """The chain-rule gradient of the disk renderer against central finite
    differences of the renderer itself (FP64), for a random linear functional."""
    N, S, rmax = 33, 0.5, 8.0
    rng = np.random.default_rng(21)
    dZ = rng.standard_normal(N * N)
    g = O.render_disk_grad(N, S, rmax, THETA, dZ)
    for k in range(5):
        h = 1e-6 * max(abs(THETA[k]), 1e-3)
        tp, tm = list(THETA), list(THETA)
        tp[k] += h
        tm[k] -= h
        fd = (dZ @ O.render_disk(N, S, rmax, tp) - dZ @ O.render_disk(N, S, rmax, tm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * (abs(fd) + abs(g[k])) + 1e-30, (k, fd, g[k])


def test_disk_face_on_is_radial_and_peaks_near_r0():
    N, S = 65, 0.25
    th = (0.0, 5.0, 0.6, -1.0, 1.0)
    Z = O.render_disk(N, S, 100.0, th).reshape(N, N)
    assert np.allclose(Z, Z.T) and np.allclose(Z, Z[::-1, :])
    x, y, r, _, _ = O.scene_geometry(N, S)
    rr = r.reshape(N, N)
    peak = rr.ravel()[np.argmax(Z)]
    # maximum of u^g exp(-(rho-r0)^2/2w^2): g/rho = (rho - r0)/w^2
    rho_star = (5.0 + math.sqrt(25.0 + 4 * 0.36 * -1.0)) / 2
    assert abs(peak - rho_star) <= S


def test_chi2_pins():
    """The misfit's definition pinned by what it must satisfy: zero at
    D = K S (with a zero gradient), a one-pixel value worked by hand, the
    gradient against FP64 central differences of the loss, and 1/var
    scaling."""
    S = np.array([2.0, 0.5, 1.25])
    K = 4.0
    L, g = O.chi2(S, K * S, np.ones(3), K)
    assert L == 0.0 and np.all(g == 0.0)
    # one pixel: (4*3 - 10)^2 / 2 = 2, gradient 2*4*(12 - 10)/2 = 8
    L1, g1 = O.chi2([3.0], [10.0], [2.0], 4.0)
    assert L1 == 2.0 and g1[0] == 8.0
    rng = np.random.default_rng(5)
    S = rng.random(7)
    D = rng.random(7) * 4.0
    V = 0.5 + rng.random(7)
    L, g = O.chi2(S, D, V, 3.0)
    for i in range(7):
        h = 1e-6
        Sp, Sm = S.copy(), S.copy()
        Sp[i] += h
        Sm[i] -= h
        fd = (O.chi2(Sp, D, V, 3.0)[0] - O.chi2(Sm, D, V, 3.0)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
    L2, g2 = O.chi2(S, D, 2.0 * V, 3.0)
    assert abs(L2 - 0.5 * L) <= 1e-15 * L and np.allclose(g2, 0.5 * g, rtol=1e-15, atol=0)
