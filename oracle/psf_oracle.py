"""FP64 reference ("oracle") for the field-dependent PSF operator.

TEST INFRASTRUCTURE ONLY.  This module is imported by the test-suite, by the
package's ``smoke()`` check and by the benchmark's CPU-baseline leg, and by
nothing else: the product path (the HIP library and its Python binding) never
calls it and shares no code with it.

It follows Milani & Douglas, "Faster imaging simulation through complex
systems: a coronagraphic example" (arXiv 2106.09122):

* Sec. 2 and Eqs. (2)-(3): the scene meshgrid of pixel-centre offsets,
  the polar conversion of each field point, radial interpolation of the
  off-axis PSF datacube (linear or nearest) and rotation of the result to the
  field point's position angle; one flattened PSF per scene pixel.
* Sec. 3, Eqs. (4)-(6): the library matrix A = [I_1 ... I_{N^2}] with one
  column per scene pixel, and the simulated image S = A Z.

Everything is plain numpy in float64, one column at a time, in the order the
paper describes.  Inputs are the same float32 cube values (promoted exactly)
and float64 radii the GPU receives.

Readings taken where the paper is silent or garbled (each one is listed in
the repository's design notes):

* meshgrid centres are (q - (N-1)/2) * S for column q and (p - (N-1)/2) * S
  for row p: x follows the column index, y the row index, both flattened
  row-major;
* the polar angle is carried as (cos, sin) = (x/r, y/r), and (1, 0) at r = 0
  (the value atan2 gives there);
* rotation turns the +x-axis PSF so that its core lands on the field point
  (with y increasing with row index), about the array centre ((n-1)/2,
  (n-1)/2), keeping the n x n frame; the rotated image is sampled bilinearly
  with zero padding outside the array, or (the paper's rotate() default) by
  the cubic B-spline that interpolates the PSF extended by zeros;
* offsets beyond the last sample either hold the last PSF (``clamp``) or give
  an all-zero column (``zero``); offsets below the first sample hold the
  first PSF;
* optionally (flux="preserve") each column is rescaled to the total of the
  radially interpolated PSF before rotation;
* nearest-neighbour radial interpolation rounds ties to the lower sample;
* the operator applies no normalisation of its own (Sec. 3 leaves PSF
  normalisation to the user); column sums are reported instead.

The per-column power-of-two scaled 16-bit storage (``pow2_exponents``,
``round_to_format``) is not in the paper, which stores float64; it is the
reduced-precision form of the same matrix, and its exact FP64 definition is
given here so the GPU's rounding error can be measured against it.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "scene_geometry", "radial_bracket", "interpolate_radial", "rotate_bilinear",
    "spline_prefilter", "spline_prefilter_1d", "spline_coefficients", "bspline3", "rotate_cubic",
    "library_column", "build_library", "column_sums", "apply", "apply_adjoint",
    "apply_batched", "pow2_exponents", "column_max_bound", "round_to_format",
    "quantize_library", "scale_exponent", "ZERO_COLUMN_EXPONENT", "render_disk", "render_disk_grad",
    "chi2",
]


# ------------------------------------------------------------------ a1 ----
def scene_geometry(N: int, S: float):
    """Pixel-centre offsets and polar form of every scene pixel.

    Sec. 2, Eqs. (2)-(3): a meshgrid running over the N pixels with a half
    pixel shift, scaled by the scene pixel scale S; flattened so that scene
    pixel (row p, col q) is field point j = p*N + q.  The polar conversion
    (Sec. 2, "standard 2D arctangent") is kept as r and the unit vector
    (cos, sin) = (x/r, y/r).

    Returns x, y, r, ct, st as float64 arrays of length N*N.
    """
    N = int(N)
    S = float(S)
    C = (N - 1) / 2.0
    p, q = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(N, dtype=np.float64),
                       indexing="ij")
    x = ((q - C) * S).ravel()
    y = ((p - C) * S).ravel()
    r = np.sqrt(x * x + y * y)
    ct = np.ones_like(r)
    st = np.zeros_like(r)
    nz = r > 0
    ct[nz] = x[nz] / r[nz]
    st[nz] = y[nz] / r[nz]
    return x, y, r, ct, st


# ------------------------------------------------------------------ a2 ----
def radial_bracket(r: float, radii: np.ndarray, interp: str = "linear", oob: str = "clamp"):
    """Radial sample pair and weight for one offset r.

    Sec. 2: the interpolating function, set up on the datacube of PSFs with
    offsets along one axis, returns the PSF interpolated (linear or nearest)
    to the offset r.  Returns (k, w, zero): Q = (1-w) P_k + w P_{k+1}; if
    ``zero`` the column is identically zero.
    """
    radii = np.asarray(radii, dtype=np.float64)
    K = radii.size
    if K == 1:
        return 0, 0.0, False
    if r <= radii[0]:
        return 0, 0.0, False
    if r >= radii[K - 1]:
        if oob == "zero" and r > radii[K - 1]:
            return K - 2, 0.0, True
        return K - 2, 1.0, False
    # largest k with radii[k] <= r  (0 <= k <= K-2 here)
    k = int(np.searchsorted(radii, r, side="right")) - 1
    lo, hi = radii[k], radii[k + 1]
    if interp == "nearest":
        # ties go to the lower sample
        return k, (1.0 if (r - lo) > (hi - r) else 0.0), False
    return k, (r - lo) / (hi - lo), False


def interpolate_radial(cube: np.ndarray, k: int, w: float) -> np.ndarray:
    """Q = (1-w) P_k + w P_{k+1} in float64 (Sec. 2, linear interpolation in
    offset at the integer pixel nodes of the datacube)."""
    P = np.asarray(cube, dtype=np.float64)
    if P.shape[0] == 1:
        return P[0].copy()
    return (1.0 - w) * P[k] + w * P[k + 1]


# ------------------------------------------------------------------ a3 ----
def rotate_bilinear(Q: np.ndarray, ct: float, st: float) -> np.ndarray:
    """Rotate an n x n PSF about its centre so that a feature on +x moves to
    position angle theta (cos theta = ct, sin theta = st), sampling bilinearly
    with zero padding (Sec. 2, the rotation step).

    Output pixel (a, b) has offset u = (b - c, a - c) from the centre
    c = (n-1)/2; it samples Q at c + R(-theta) u, i.e. at column
    c + ct*ux + st*uy and row c - st*ux + ct*uy.
    """
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[0]
    c = (n - 1) / 2.0
    a, b = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")
    ux = b - c
    uy = a - c
    sx = ct * ux + st * uy
    sy = (-st) * ux + ct * uy
    col = c + sx
    row = c + sy
    c0 = np.floor(col)
    r0 = np.floor(row)
    fx = col - c0
    fy = row - r0
    c0 = c0.astype(np.int64)
    r0 = r0.astype(np.int64)

    def tap(rr, cc):
        ok = (rr >= 0) & (rr < n) & (cc >= 0) & (cc < n)
        v = np.zeros_like(fx)
        v[ok] = Q[rr[ok], cc[ok]]
        return v

    return ((1.0 - fy) * (1.0 - fx) * tap(r0, c0)
            + (1.0 - fy) * fx * tap(r0, c0 + 1)
            + fy * (1.0 - fx) * tap(r0 + 1, c0)
            + fy * fx * tap(r0 + 1, c0 + 1))


# ------------------------------------------ a3, cubic-spline rotation ----
# The paper rotates with SciPy's rotate(), whose default interpolation is a
# cubic spline.  The PSF is extended by zeros outside its frame; the spline
# that interpolates the extended image is f(x) = sum_m c_m beta3(x - m) with
# beta3 the cubic B-spline.  Its coefficients are computed on the frame
# padded by SPLINE_PAD zero pixels per side with the exact recursive filter
# for a mirror-symmetric extension of that padded array (the pole is
# sqrt(3) - 2, so the padding leaves the frame's own coefficients within
# (2 - sqrt(3))^12 ~ 1e-7 of the infinite-extension values), and taken as zero
# beyond the padded array.
SPLINE_PAD = 12
_SPLINE_POLE = math.sqrt(3.0) - 2.0


def spline_prefilter(a, axis: int = 0) -> np.ndarray:
    """Cubic B-spline interpolation coefficients of the samples in `a` along
    `axis`, under a mirror-symmetric extension: gain 6, then one causal and
    one anticausal first-order recursion with pole z = sqrt(3) - 2 (the
    standard B-spline interpolation filter).  The causal start value sums
    the mirrored signal over one full period, so the result is exact for
    the periodic mirror extension.  Every line along `axis` is filtered
    independently (the recursion runs over `axis`, vectorised across the
    other axes)."""
    z = _SPLINE_POLE
    c = 6.0 * np.moveaxis(np.asarray(a, dtype=np.float64), axis, 0)
    N = c.shape[0]
    if N == 1:
        return np.moveaxis(c / 6.0, 0, axis)
    k = np.arange(1, N - 1).reshape((-1,) + (1,) * (c.ndim - 1))
    start = (c[0] + z ** (N - 1) * c[N - 1]
             + np.sum((z ** k + z ** (2 * N - 2 - k)) * c[1:N - 1], axis=0)) / (1.0 - z ** (2 * N - 2))
    cp = np.empty_like(c)
    cp[0] = start
    for i in range(1, N):
        cp[i] = c[i] + z * cp[i - 1]
    cm = np.empty_like(c)
    cm[N - 1] = (z / (z * z - 1.0)) * (cp[N - 1] + z * cp[N - 2])
    for i in range(N - 2, -1, -1):
        cm[i] = z * (cm[i + 1] - cp[i])
    return np.moveaxis(cm, 0, axis)


def spline_prefilter_1d(s) -> np.ndarray:
    """spline_prefilter of a single line."""
    return spline_prefilter(np.asarray(s, dtype=np.float64), 0)


def spline_coefficients(Q, pad: int = SPLINE_PAD) -> np.ndarray:
    """Coefficients of the cubic spline interpolating Q extended by zeros:
    Q padded with `pad` zero pixels per side, filtered along each column,
    then along each row.  Returns float64 [(n + 2 pad)][(n + 2 pad)]."""
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[0]
    P = np.zeros((n + 2 * pad, n + 2 * pad))
    P[pad:pad + n, pad:pad + n] = Q
    return spline_prefilter(spline_prefilter(P, 0), 1)


def bspline3(t) -> np.ndarray:
    """The centred cubic B-spline: 2/3 - t^2 + |t|^3/2 on |t| < 1,
    (2 - |t|)^3 / 6 on 1 <= |t| < 2, 0 beyond."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(t < 1.0, 2.0 / 3.0 - t * t + t * t * t / 2.0,
                    np.where(t < 2.0, (2.0 - t) ** 3 / 6.0, 0.0))


def rotate_cubic(Q: np.ndarray, ct: float, st: float, pad: int = SPLINE_PAD) -> np.ndarray:
    """Rotate like rotate_bilinear (same source coordinates), sampling the
    cubic spline of Q extended by zeros: the 4 x 4 coefficients around the
    source point, weighted by beta3 of the distances along rows and columns;
    coefficients outside the padded array count as zero."""
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[0]
    c = (n - 1) / 2.0
    C = spline_coefficients(Q, pad)
    Mp = n + 2 * pad
    a, b = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")
    ux = b - c
    uy = a - c
    sx = ct * ux + st * uy
    sy = (-st) * ux + ct * uy
    col = c + sx + pad  # coordinates in the padded array
    row = c + sy + pad
    r0 = np.floor(row).astype(np.int64)
    c0 = np.floor(col).astype(np.int64)
    out = np.zeros_like(col)
    for dr in (-1, 0, 1, 2):
        rr = r0 + dr
        wy = bspline3(row - rr)
        for dc in (-1, 0, 1, 2):
            cc = c0 + dc
            wx = bspline3(col - cc)
            ok = (rr >= 0) & (rr < Mp) & (cc >= 0) & (cc < Mp)
            v = np.zeros_like(col)
            v[ok] = C[rr[ok], cc[ok]]
            out += wy * wx * v
    return out


def library_column(cube, radii, r, ct, st, interp="linear", oob="clamp",
                   rotate="bilinear", flux="none") -> np.ndarray:
    """One library column I_j: radial interpolation, rotation, flattening
    (Sec. 2, one iteration of the field-point loop).

    flux="preserve" rescales the column so that it sums to the flux of the
    radially interpolated PSF Q before rotation (the part of Q that the
    rotation carries out of the frame, or the spline's overshoot, no longer
    changes the column's total); a column that sums to zero is left as is."""
    cube = np.asarray(cube)
    n = cube.shape[1]
    k, w, zero = radial_bracket(r, radii, interp, oob)
    if zero:
        return np.zeros(n * n, dtype=np.float64)
    Q = interpolate_radial(cube, k, w)
    if rotate == "cubic":
        col = rotate_cubic(Q, ct, st).ravel()
    elif rotate == "bilinear":
        col = rotate_bilinear(Q, ct, st).ravel()
    else:
        raise ValueError("rotate must be 'bilinear' or 'cubic'")
    if flux == "preserve":
        tau = col.sum()
        if tau != 0.0:
            col = col * (Q.sum() / tau)
    elif flux != "none":
        raise ValueError("flux must be 'none' or 'preserve'")
    return col


def build_library(cube, radii, N: int, S: float, interp: str = "linear", oob: str = "clamp",
                  columns=None, rotate: str = "bilinear", flux: str = "none") -> np.ndarray:
    """The library matrix A (Sec. 3, Eqs. (4)-(5)): n^2 rows, one column per
    scene pixel, column j the flattened interpolated-and-rotated PSF of field
    point j.  ``columns`` selects a subset of j (returned in that order).
    Returns float64 [n*n][len(columns)]."""
    cube = np.asarray(cube)
    if cube.ndim != 3 or cube.shape[1] != cube.shape[2]:
        raise ValueError("cube must be [K][n][n]")
    radii = np.asarray(radii, dtype=np.float64)
    if radii.size != cube.shape[0]:
        raise ValueError("one radius per PSF")
    n = cube.shape[1]
    _, _, r, ct, st = scene_geometry(N, S)
    cols = np.arange(N * N) if columns is None else np.asarray(columns, dtype=np.int64)
    A = np.empty((n * n, cols.size), dtype=np.float64)
    for t, j in enumerate(cols):
        A[:, t] = library_column(cube, radii, r[j], ct[j], st[j], interp, oob, rotate, flux)
    return A


# ---------------------------------------------------------- a5, a6, a7 ----
def column_sums(A: np.ndarray) -> np.ndarray:
    """tau_j = sum_i A_ij: the throughput of each library column."""
    return np.asarray(A, dtype=np.float64).sum(axis=0)


def apply(A: np.ndarray, Z) -> np.ndarray:
    """Simulated image S = A Z (Sec. 3, Eq. (6)), float64."""
    return np.asarray(A, dtype=np.float64) @ np.asarray(Z, dtype=np.float64)


def apply_adjoint(A: np.ndarray, g) -> np.ndarray:
    """G = A^T g, the adjoint of the simulation (gradient of <g, A Z> in Z)."""
    return np.asarray(A, dtype=np.float64).T @ np.asarray(g, dtype=np.float64)


def apply_batched(A: np.ndarray, Zb) -> np.ndarray:
    """Images of B scenes at once: out[b] = A Z_b.  Zb is [B][N*N]."""
    Zb = np.asarray(Zb, dtype=np.float64)
    return (np.asarray(A, dtype=np.float64) @ Zb.T).T


# ------------------------------------------------------------------ a4 ----
# An identically zero column has no scale of its own.  Its exponent is chosen
# so that every finite value times 2**e underflows to exactly 0, in float32 and
# in float64: a scene value at that column (which multiplies only zeros) then
# cannot set the per-scene scale of the 16-bit product or overflow the format.
ZERO_COLUMN_EXPONENT = -16384


def scale_exponent(m: float) -> int:
    """Power-of-two exponent e with m * 2**-e in [2**14, 2**15) for m > 0,
    and ZERO_COLUMN_EXPONENT for m == 0."""
    if m == 0.0:
        return ZERO_COLUMN_EXPONENT
    _, E = math.frexp(m)  # m = f * 2**E, f in [0.5, 1)
    return E - 15


def column_max_bound(cube, radii, N: int, S: float, interp="linear", oob="clamp",
                     rotate="bilinear") -> np.ndarray:
    """Per-column upper bound on max_i |A_ij| that needs no column values:
    (1-w) m_k + w m_{k+1}.  Bilinear rotation is a convex combination of Q's
    pixels (or zero), so with m_k = max(P_k) (the cube is non-negative) the
    column never exceeds it.  The cubic spline is a convex combination of
    coefficients, and Q's coefficients are (1-w) C_k + w C_{k+1} (the
    prefilter is linear), so m_k = max |C_k| bounds it."""
    cube = np.asarray(cube, dtype=np.float64)
    if rotate == "cubic":
        pmax = np.array([np.abs(spline_coefficients(P)).max() for P in cube])
    else:
        pmax = cube.reshape(cube.shape[0], -1).max(axis=1)
    _, _, r, _, _ = scene_geometry(N, S)
    out = np.empty(r.size, dtype=np.float64)
    for j in range(r.size):
        k, w, zero = radial_bracket(r[j], radii, interp, oob)
        if zero:
            out[j] = 0.0
        elif cube.shape[0] == 1:
            out[j] = pmax[0]
        else:
            out[j] = (1.0 - w) * pmax[k] + w * pmax[k + 1]
    return out


def pow2_exponents(bound: np.ndarray) -> np.ndarray:
    """Per-column exponents e_j = scale_exponent(bound_j) (int32)."""
    return np.array([scale_exponent(float(b)) for b in np.asarray(bound, dtype=np.float64)],
                    dtype=np.int32)


def round_to_format(v, fmt: str) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 or IEEE binary16 value
    (round to nearest, ties to even), returned as float64.

    binary16: 11 significant bits, normal exponents down to -14 and
    subnormals spaced 2**-24, largest finite 65504.  bfloat16: 8
    significant bits with the float32 exponent range (subnormals spaced
    2**-133)."""
    v = np.asarray(v, dtype=np.float64)
    if fmt == "fp16":
        p, emin, vmax = 11, -14, 65504.0
    elif fmt == "bf16":
        p, emin, vmax = 8, -126, float(np.ldexp(255.0 / 128.0, 127))
    else:
        raise ValueError(fmt)
    out = np.zeros_like(v)
    a = np.abs(v)
    nz = a > 0
    _, E = np.frexp(a[nz])  # a = f * 2**E, f in [0.5, 1): leading bit at 2**(E-1)
    lead = np.maximum(E - 1, emin)
    quantum = np.ldexp(1.0, lead - (p - 1))
    q = np.rint(a[nz] / quantum) * quantum  # rint: ties to even
    q = np.where(q > vmax, np.inf, q)  # rounded past the largest finite value
    out[nz] = np.copysign(q, v[nz])
    return out


def quantize_library(A: np.ndarray, e: np.ndarray, fmt: str) -> np.ndarray:
    """Mantissa matrix M_ij = RN(A_ij * 2**-e_j) in the 16-bit format, as
    float64 (exact)."""
    A = np.asarray(A, dtype=np.float64)
    # ldexp scales exactly (a zero column stays 0 at any exponent)
    return round_to_format(np.ldexp(A, -np.asarray(e, dtype=np.int64)[None, :]), fmt)


# ------------------------------------------------ fitting model (disk) ----
# A smooth parametric exozodi disk, the model fitted through the operator
# (the gradient analogue of the retrieval the paper's conclusions plan).
# Parameters theta = (incl [rad], r0, width, gamma, flux):
#   rho = sqrt(x^2 + (y / cos incl)^2)       (deprojected radius, x on the major axis)
#   Z   = flux * (rho/r0)^gamma * exp(-(rho - r0)^2 / (2 width^2))
# on the scene meshgrid of Eqs. (2)-(3); Z = 0 where rho == 0 or where the sky
# radius exceeds rmax (the paper masks scenes outside the working angle).

def render_disk(N: int, S: float, rmax: float, theta) -> np.ndarray:
    """Disk scene Z (float64 [N*N]) for parameters theta."""
    incl, r0, w, g, F = (float(t) for t in theta)
    x, y, r, _, _ = scene_geometry(N, S)
    ci = math.cos(incl)
    rho = np.sqrt(x * x + (y / ci) ** 2)
    Z = np.zeros_like(rho)
    m = (rho > 0) & (r <= rmax)
    u = rho[m] / r0
    Z[m] = F * u**g * np.exp(-((rho[m] - r0) ** 2) / (2 * w * w))
    return Z


def render_disk_grad(N: int, S: float, rmax: float, theta, dZ) -> np.ndarray:
    """Chain rule through the renderer: sum_j dZ_j * dZ_j/dtheta (float64 [5])."""
    incl, r0, w, g, F = (float(t) for t in theta)
    x, y, r, _, _ = scene_geometry(N, S)
    ci, si = math.cos(incl), math.sin(incl)
    rho = np.sqrt(x * x + (y / ci) ** 2)
    m = (rho > 0) & (r <= rmax)
    rho, y, d = rho[m], y[m], np.asarray(dZ, dtype=np.float64)[m]
    Z = F * (rho / r0) ** g * np.exp(-((rho - r0) ** 2) / (2 * w * w))
    dZ_drho = Z * (g / rho - (rho - r0) / (w * w))
    drho_dincl = y * y * si / (ci**3 * rho)
    out = np.empty(5)
    out[0] = np.sum(d * dZ_drho * drho_dincl)
    out[1] = np.sum(d * Z * (-g / r0 + (rho - r0) / (w * w)))
    out[2] = np.sum(d * Z * (rho - r0) ** 2 / w**3)
    out[3] = np.sum(d * Z * np.log(rho / r0))
    out[4] = np.sum(d * Z / F)
    return out


def chi2(S, D, var, K: float):
    """Misfit of a simulated image for Gaussian errors, the quantity the
    retrieval the paper's conclusions plan would minimise:
    L = sum_i (K S_i - D_i)^2 / var_i, with its gradient in the image
    dL/dS_i = 2 K (K S_i - D_i) / var_i.  float64; the sum is exactly rounded
    (math.fsum).  Returns (L, gradient)."""
    r = float(K) * np.asarray(S, dtype=np.float64) - np.asarray(D, dtype=np.float64)
    v = np.asarray(var, dtype=np.float64)
    return math.fsum((r * r / v).tolist()), (2.0 * float(K)) * r / v
