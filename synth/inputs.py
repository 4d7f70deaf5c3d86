"""Seeded synthetic workloads shaped like the paper's inputs.

The paper's data (IPAC/PROPER off-axis PSF cubes, ZODIPIC exozodi scenes;
Sec. 2 and Sec. 4.1) are not available, so these generators stand in for
them with the same shapes and value ranges:

* ``psf_cube`` -- a datacube of off-axis PSFs with sources offset along +x
  (Sec. 2: "a datacube of PSFs with angular offsets along one dimension").
  Each PSF is a Fraunhofer image of a circular pupil with seeded low-order
  Zernike phase errors, computed with an explicit matrix DFT so the optical
  axis lands on the array centre ((n-1)/2, (n-1)/2), times a coronagraph-like
  throughput curve that is 0 inside 3 lambda/D and 1 beyond 4 lambda/D.
* ``ring_scene`` -- an inclined power-law dust ring (stand-in for a ZODIPIC
  scene, Sec. 2 / Fig. 2), masked outside the largest sampled offset the way
  the paper masks outside the outer working angle.
* ``planets`` -- point sources snapped to scene pixels.

Angles are in units of lambda0/D throughout.  Every draw comes from
``numpy.random.default_rng([210609122, config, stream])`` so each workload is
reproducible bit for bit.  Nothing here implements the operator itself.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = 210609122

# random streams
STREAM_ABERR, STREAM_DISK, STREAM_PLANETS, STREAM_NOISE, STREAM_SUBSAMPLE, STREAM_BATCH = range(6)


def rng_for(config: int, stream: int) -> np.random.Generator:
    """PCG64 generator for (config, stream)."""
    return np.random.default_rng([SEED_ROOT, int(config), int(stream)])


# ---------------------------------------------------------------- radii ----
def radii_linspace(K: int, rmax: float = 8.0) -> np.ndarray:
    """K offsets evenly spaced on [0, rmax] (inclusive), FP64."""
    return np.linspace(0.0, rmax, int(K))


def radii_nonuniform() -> np.ndarray:
    """Offsets with the IPAC HLC cube's sampling pattern (Sec. 2): 0.06 below
    4, 0.5 between 4 and 9, 0.25 between 9 and 11 (lambda/D).  The count that
    results (86) differs by one from the 85 the paper quotes; the pattern,
    not the count, is what matters for a non-uniform bracket search."""
    a = np.arange(0.0, 4.0, 0.06)
    b = np.arange(4.0, 9.0, 0.5)
    c = np.arange(9.0, 11.0 + 1e-9, 0.25)
    return np.concatenate([a, b, c]).astype(np.float64)


# ------------------------------------------------------------ PSF cube -----
def _zernike_noll(j: int, rho: np.ndarray, th: np.ndarray) -> np.ndarray:
    """Noll-normalised Zernike polynomials 4..11 on the unit disk."""
    if j == 4:
        return np.sqrt(3.0) * (2 * rho**2 - 1)
    if j == 5:
        return np.sqrt(6.0) * rho**2 * np.sin(2 * th)
    if j == 6:
        return np.sqrt(6.0) * rho**2 * np.cos(2 * th)
    if j == 7:
        return np.sqrt(8.0) * (3 * rho**3 - 2 * rho) * np.sin(th)
    if j == 8:
        return np.sqrt(8.0) * (3 * rho**3 - 2 * rho) * np.cos(th)
    if j == 9:
        return np.sqrt(8.0) * rho**3 * np.sin(3 * th)
    if j == 10:
        return np.sqrt(8.0) * rho**3 * np.cos(3 * th)
    if j == 11:
        return np.sqrt(5.0) * (6 * rho**4 - 6 * rho**2 + 1)
    raise ValueError(j)


def throughput(r: np.ndarray) -> np.ndarray:
    """Coronagraph-like throughput: 0 for r <= 3, sin^2 ramp on (3, 4), 1 beyond."""
    r = np.asarray(r, dtype=np.float64)
    t = np.where(r >= 4.0, 1.0, np.sin(np.pi * (r - 3.0) / 2.0) ** 2)
    return np.where(r <= 3.0, 0.0, t)


def psf_cube(n: int, s: float, radii, *, rng: np.random.Generator | None = None,
             config: int = 0, npup: int = 128, wavelength_ratio: float = 1.0,
             aberration_rms: float = 0.02, apply_throughput: bool = True) -> np.ndarray:
    """Off-axis PSF datacube, float32 [K][n][n] (k, row, col).

    n: PSF side in pixels; s: PSF pixel scale in lambda0/D; radii: source
    offsets (lambda0/D) along +x.  ``wavelength_ratio`` = lambda/lambda0
    dilates the PSF, scales the phase by lambda0/lambda and evaluates the
    throughput at r*lambda0/lambda.  The unaberrated on-axis peak at lambda0
    is 1.  The result is cast to float32 once, at the end.
    """
    if rng is None:
        rng = rng_for(config, STREAM_ABERR)
    radii = np.asarray(radii, dtype=np.float64)
    ell = float(wavelength_ratio)
    coeffs = rng.normal(0.0, aberration_rms, size=8)  # Noll 4..11, waves at lambda0
    xp = (np.arange(npup) - (npup - 1) / 2.0) / npup  # pupil coords in units of D
    X, Y = np.meshgrid(xp, xp)
    rho = np.hypot(X, Y) / 0.5
    th = np.arctan2(Y, X)
    pupil = (rho <= 1.0).astype(np.float64)
    phase = np.zeros_like(X)
    for idx, j in enumerate(range(4, 12)):
        phase += coeffs[idx] * _zernike_noll(j, rho, th)
    phase = phase / ell
    field0 = pupil * np.exp(2j * np.pi * phase)
    norm = pupil.sum() ** 2
    c = (n - 1) / 2.0
    u = (np.arange(n) - c) * s / ell  # focal-plane coords in lambda/D at this wavelength
    Wu = np.exp(-2j * np.pi * np.outer(u, xp))  # [n][npup]
    out = np.empty((radii.size, n, n), dtype=np.float64)
    for k, rk in enumerate(radii):
        tilt = np.exp(2j * np.pi * X * (rk / ell))
        E = Wu @ (field0 * tilt) @ Wu.T  # rows: v (y), cols: u (x)
        I = (E.real**2 + E.imag**2) / norm
        if apply_throughput:
            I = I * throughput(rk / ell)
        out[k] = I
    return out.astype(np.float32)


# -------------------------------------------------------------- scenes -----
def _pixel_offsets(N: int, S: float):
    """Scene pixel-centre offsets for *rendering* a scene (x = column, y = row)."""
    t = (np.arange(N) - (N - 1) / 2.0) * S
    x = np.broadcast_to(t[None, :], (N, N))
    y = np.broadcast_to(t[:, None], (N, N))
    return x, y


def ring_scene(N: int, S: float, *, incl_deg: float = 60.0, r_in: float = 3.0,
               r_out: float = 9.0, gamma: float = -1.5, total_flux: float = 1e-7,
               rmax_mask: float | None = None) -> np.ndarray:
    """Inclined power-law ring, float32 [N][N] (row, col).

    Deprojected radius rho = sqrt(x^2 + (y/cos i)^2) with the major axis on
    x; brightness rho**gamma for r_in <= rho <= r_out, normalised to
    ``total_flux`` (star = 1).  Pixels with sky radius > rmax_mask are zeroed
    (the paper masks its scenes outside the outer working angle)."""
    x, y = _pixel_offsets(N, S)
    ci = np.cos(np.deg2rad(incl_deg))
    rho = np.sqrt(x**2 + (y / ci) ** 2)
    img = np.where((rho >= r_in) & (rho <= r_out), np.power(np.maximum(rho, 1e-12), gamma), 0.0)
    if rmax_mask is not None:
        img = np.where(np.hypot(x, y) > rmax_mask, 0.0, img)
    tot = img.sum()
    if tot > 0:
        img = img * (total_flux / tot)
    return img.astype(np.float32)


def planets(N: int, S: float, count: int, rng: np.random.Generator, *,
            r_range=(3.5, 7.5), contrast=(1e-9, 1e-7)):
    """``count`` point sources: radius ~ U(r_range), position angle ~ U(0, 2pi),
    snapped to the nearest scene pixel; contrast log-uniform in ``contrast``.
    Returns a list of (row, col, flux)."""
    out = []
    c = (N - 1) / 2.0
    for _ in range(int(count)):
        r = rng.uniform(*r_range)
        pa = rng.uniform(0.0, 2 * np.pi)
        f = float(np.exp(rng.uniform(np.log(contrast[0]), np.log(contrast[1]))))
        col = int(np.clip(np.rint(c + r * np.cos(pa) / S), 0, N - 1))
        row = int(np.clip(np.rint(c + r * np.sin(pa) / S), 0, N - 1))
        out.append((row, col, f))
    return out


def add_planets(scene: np.ndarray, pl) -> np.ndarray:
    out = scene.astype(np.float64).copy()
    for row, col, f in pl:
        out[row, col] += f
    return out.astype(np.float32)


def random_ring_params(rng: np.random.Generator):
    """Seeded disk parameters: i ~ U(0, 80 deg), r0 ~ U(3, 9), ring
    [0.8 r0, 1.2 r0], gamma ~ U(-2, -1)."""
    inc = rng.uniform(0.0, 80.0)
    r0 = rng.uniform(3.0, 9.0)
    g = rng.uniform(-2.0, -1.0)
    return dict(incl_deg=inc, r_in=0.8 * r0, r_out=1.2 * r0, gamma=g)


def scene_batch(N: int, S: float, B: int, *, config: int, rmax_mask: float) -> np.ndarray:
    """B seeded ring scenes, float32 [B][N*N]."""
    rng = rng_for(config, STREAM_BATCH)
    out = np.empty((B, N * N), dtype=np.float32)
    for b in range(B):
        out[b] = ring_scene(N, S, rmax_mask=rmax_mask, **random_ring_params(rng)).ravel()
    return out


# ------------------------------------------------------------- configs -----
CONFIGS = {
    # plain method at 32x32, 0.5 lambda/D per pixel, 16 PSFs over 0..8
    1: dict(n=32, N=32, s=0.5, S=0.5, K=16, planets=2),
    # single-scene HBM-bound matvec at 128x128 (16384 x 16384 library)
    2: dict(n=128, N=128, s=0.125, S=0.125, K=64, planets=5),
    # differentiation workload uses the 128x128 library
    4: dict(n=128, N=128, s=0.125, S=0.125, K=64, planets=0),
    # large library 256x256 (65536 x 65536)
    5: dict(n=256, N=256, s=0.0625, S=0.0625, K=128, planets=0),
    # the paper's own shape (its IPAC set, Sec. 4): 128x128 PSFs at 0.2 lambda/D
    # with the IPAC offset pattern to 11 lambda/D, a 256x256 scene at
    # 3.529 mas = 0.2 * 3.529 / 10.0379 lambda/D (Eq. 1's 0.2 lambda/D =
    # 10.0379 mas): a 16384 x 65536 library
    6: dict(n=128, N=256, s=0.2, S=0.2 * 3.529 / 10.0379, K=None, planets=3),
}


def config_inputs(config: int, *, with_cube: bool = True) -> dict:
    """Cube, radii and one scene for a numbered workload.

    Returns dict(n, N, s, S, radii[K] f64, cube[K][n][n] f32, scene[N*N] f32)."""
    p = dict(CONFIGS[config])
    radii = radii_nonuniform() if p["K"] is None else radii_linspace(p["K"], 8.0)
    out = dict(n=p["n"], N=p["N"], s=p["s"], S=p["S"], radii=radii)
    if with_cube:
        out["cube"] = psf_cube(p["n"], p["s"], radii, rng=rng_for(config, STREAM_ABERR))
    scene = ring_scene(p["N"], p["S"], incl_deg=60.0, r_in=3.0, r_out=9.0, gamma=-1.5,
                       rmax_mask=float(radii[-1]))
    if p["planets"]:
        pl = planets(p["N"], p["S"], p["planets"], rng_for(config, STREAM_PLANETS))
        scene = add_planets(scene, pl)
    out["scene"] = scene.ravel()
    return out


# ------------------------------------------------------ fitting data -------
DISK_TRUE = (1.0471975511965976, 5.0, 1.2, -1.4, 3e-8)  # (60 deg, r0, width, gamma, flux)
DISK_START = (0.9, 5.6, 1.5, -1.1, 2e-8)


def noisy_counts(image, peak_counts: float, rng: np.random.Generator, read_noise: float = 3.0):
    """Detector counts for a simulated image: Poisson(K * image) + N(0, read_noise^2),
    with K chosen so the brightest pixel expects `peak_counts`.  Returns
    (counts float64, K, variance estimate max(counts, 1) + read_noise^2)."""
    image = np.asarray(image, dtype=np.float64)
    K = peak_counts / image.max()
    lam = np.clip(K * image, 0.0, None)
    counts = rng.poisson(lam).astype(np.float64) + rng.normal(0.0, read_noise, size=lam.shape)
    var = np.maximum(counts, 1.0) + read_noise**2
    return counts, K, var


# ------------------------------------------------ mixed-size workload ------
MIXED_SIZES = (64, 96, 128)
MIXED_WAVELENGTHS = tuple(0.95 + 0.01 * w for w in range(11))  # lambda/lambda0, 575 nm centre, 10% band


def mixed_workload(B: int = 256, sizes=MIXED_SIZES, wavelengths=MIXED_WAVELENGTHS, config: int = 3):
    """Scenes of mixed sizes and wavelengths, each simulated with the library of
    its (size, wavelength).  Libraries: n = N, s = S = 16/n lambda0/D, K = n/2
    offsets on [0, 8] lambda0/D, PSFs dilated by lambda/lambda0.  Scenes: seeded
    ring disks masked beyond 8 lambda0/D.

    Returns (libs, scene_lib, scenes): libs is a list of dict(n, N, S, radii,
    cube, wavelength_ratio); scene_lib[b] indexes libs; scenes[b] is float32
    [N*N] of that library's N."""
    rng = rng_for(config, STREAM_BATCH)
    libs, index = [], {}
    aberr = rng_for(config, STREAM_ABERR)
    seeds = aberr.integers(0, 2**31, size=len(sizes))
    for si, n in enumerate(sizes):
        for ell in wavelengths:
            radii = radii_linspace(n // 2, 8.0)
            s = 16.0 / n
            cube = psf_cube(n, s, radii, rng=np.random.default_rng(int(seeds[si])),
                            wavelength_ratio=ell)
            index[(n, ell)] = len(libs)
            libs.append(dict(n=n, N=n, S=s, radii=radii, cube=cube, wavelength_ratio=ell))
    scene_lib, scenes = [], []
    for _ in range(B):
        n = sizes[int(rng.integers(0, len(sizes)))]
        ell = wavelengths[int(rng.integers(0, len(wavelengths)))]
        L = index[(n, ell)]
        p = random_ring_params(rng)
        scene_lib.append(L)
        scenes.append(ring_scene(n, 16.0 / n, rmax_mask=8.0, **p).ravel())
    return libs, scene_lib, scenes
