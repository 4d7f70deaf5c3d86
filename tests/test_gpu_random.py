"""Seeded random small configurations (GPU, through the C ABI) against the FP64
oracle: every build mode and storage form on odd and tiny shapes, with the
tolerances of the dedicated tests.  Each case prints its parameters first, so a
failure names the configuration."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

U16 = {"bf16": 2.0**-8, "fp16": 2.0**-11}


def _cases(count=24, seed=2106, n_range=(2, 49), N_range=(1, 41)):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        n = int(rng.integers(*n_range))
        N = int(rng.integers(*N_range))
        K = int(rng.integers(1, 7))
        S = float(rng.uniform(0.1, 1.2))
        radii = np.concatenate([[rng.uniform(0.0, 0.5)], rng.uniform(0.05, 1.5, K - 1)]).cumsum()
        out.append(dict(
            n=n, N=N, K=K, S=S, radii=radii,
            interp=str(rng.choice(["linear", "nearest"])),
            oob=str(rng.choice(["clamp", "zero"])),
            rotate=str(rng.choice(["bilinear", "bilinear", "cubic"])),
            flux=str(rng.choice(["none", "none", "preserve"])),
            storage=str(rng.choice(["fp32", "fp32", "bf16", "fp16"])),
            B=int(rng.choice([0, 1, 2, 5, 33, 70])),
            seed=int(rng.integers(0, 2**31))))
    return out


# small PSFs (one LDS-staged pair), then large ones (a staged box per tile; the
# gather builds for 16-bit libraries beyond 256^2 that would need a float32 copy)
@pytest.mark.parametrize("case", _cases() + _cases(8, 61209, (100, 271), (1, 13)), ids=lambda c: "n{n}-N{N}-K{K}-{interp}-{oob}-{rotate}-{flux}-{storage}-B{B}".format(**c))
def test_random_configuration(case):
    import torch
    from paper_2106_09122_amd import psflib
    print("case", {k: v for k, v in case.items() if k != "radii"}, flush=True)
    c = case
    rng = np.random.default_rng(c["seed"])
    cube = (rng.random((c["K"], c["n"], c["n"])) ** 3).astype(np.float32)
    mode = dict(interp=c["interp"], oob=c["oob"], rotate=c["rotate"], flux=c["flux"])
    A = O.build_library(cube, c["radii"], c["N"], c["S"], **mode)
    lib = psflib.Library(torch.from_numpy(cube).cuda(), c["radii"], c["N"], c["S"],
                         storage=c["storage"], **mode)
    ncols, M = c["N"] ** 2, c["n"] ** 2
    cubic, f32 = c["rotate"] == "cubic", c["storage"] == "fp32"
    b = O.column_max_bound(cube, c["radii"], c["N"], c["S"], c["interp"], c["oob"], rotate=c["rotate"])
    if c["flux"] == "preserve":
        A0 = O.build_library(cube, c["radii"], c["N"], c["S"], c["interp"], c["oob"], rotate=c["rotate"])
        t0, t1 = A0.sum(axis=0), A.sum(axis=0)
        b = b * np.abs(np.where(t0 != 0, t1 / np.where(t0 != 0, t0, 1.0), 1.0))
    # entries: relative (non-negative bilinear FP32), else against the column bound;
    # 16-bit adds the format's unit and half its subnormal spacing at the column scale
    got = lib.get_columns(np.arange(ncols)).cpu().numpy().T.astype(np.float64)
    ent = 2e-6 * (np.abs(A) if not cubic else b[None, :])
    if not f32:
        e = lib.exponents().cpu().numpy().astype(np.int64)
        ent = ent + U16[c["storage"]] * (1 + 1e-5) * np.abs(A) + 2.0**-25 * np.ldexp(1.0, e)[None, :]
    assert np.all(np.abs(got - A) <= ent + 1e-300)
    # products against the oracle's: per element within u (|A||Z|) + the entry bound
    u = 1e-5 if f32 else U16[c["storage"]] + 1e-5
    Z = rng.random(ncols).astype(np.float32)
    img = lib.apply(torch.from_numpy(Z).cuda()).cpu().numpy()
    den = np.abs(A) @ Z.astype(np.float64)
    assert np.all(np.abs(img - A @ Z.astype(np.float64)) <= u * den + ent.max(axis=0) @ Z + 1e-300)
    g = rng.standard_normal(M).astype(np.float32)
    G = lib.apply_adjoint(torch.from_numpy(g).cuda()).cpu().numpy()
    gd = np.abs(g.astype(np.float64))
    assert np.all(np.abs(G - A.T @ g.astype(np.float64)) <= u * (np.abs(A).T @ gd) + ent.max(axis=0) * gd.sum() + 1e-300)
    if c["B"]:
        Zb = rng.random((c["B"], ncols)).astype(np.float32)
        out = lib.apply_batched(torch.from_numpy(Zb).cuda()).cpu().numpy()
        ref = Zb.astype(np.float64) @ A.T
        den = Zb.astype(np.float64) @ np.abs(A).T
        # the 16-bit product rounds the scenes too: 2u of the image's peak
        tol = u * den + (Zb.astype(np.float64) @ ent.max(axis=0))[:, None] if f32 else \
            2 * U16[c["storage"]] * np.max(den, axis=1, keepdims=True) + 1e-5 * den
        assert np.all(np.abs(out - ref) <= tol + 1e-300)
    lib.close()
