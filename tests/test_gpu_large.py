"""The 256 x 256 workload: 128 sampled PSFs of 256 x 256 and a 65536 x 65536
library (2^32 entries: 16 GiB in FP32, 8 GiB in 16-bit), built on the device.
The oracle computes a seeded sample of 512 columns; parity covers those
columns and the batched products of 64 scenes supported on them (so every
expected image is exact to compute), in FP32 and BF16/FP16-pow2."""
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
def c5():
    d = synth.config_inputs(5)
    N = d["N"]
    rng = synth.rng_for(5, synth.STREAM_SUBSAMPLE)
    cols = np.sort(rng.choice(N * N, 512, replace=False))
    A = O.build_library(d["cube"], d["radii"], N, d["S"], columns=cols)
    return d, cols, A


def _scenes(cols, ncols, B, seed):
    rng = np.random.default_rng(seed)
    Z = np.zeros((B, ncols), dtype=np.float32)
    Z[:, cols] = (rng.random((B, cols.size)) * 1e-8).astype(np.float32)
    return Z


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_large_library_sampled(torch, c5, storage):
    from paper_2106_09122_amd import psflib
    d, cols, Aref = c5
    N = d["N"]
    lib = psflib.Library(torch.from_numpy(d["cube"]).cuda(), d["radii"], N, d["S"], storage=storage)
    assert lib.nbytes >= N**4 * (4 if storage == "fp32" else 2)
    got = lib.get_columns(cols).cpu().numpy().T.astype(np.float64)
    if storage == "fp32":
        pos = Aref > 0
        assert np.all(got[~pos] == 0)
        assert np.max(np.abs(got[pos] - Aref[pos]) / Aref[pos]) <= LIB_REL
    else:
        u = U16[storage]
        e = lib.exponents().cpu().numpy()[cols]
        tol = (u * (1 + 1e-5) + LIB_REL) * Aref + 2.0**-25 * np.ldexp(1.0, e)[None, :]
        assert np.all(np.abs(got - Aref) <= tol)
    tau = lib.column_sums().cpu().numpy()[cols]
    np.testing.assert_allclose(tau, Aref.sum(axis=0), rtol=LIB_REL, atol=0)
    Zb = _scenes(cols, N * N, 64, 55)
    refb = Zb[:, cols].astype(np.float64) @ Aref.T
    out = lib.apply_batched(torch.from_numpy(Zb).cuda()).cpu().numpy().astype(np.float64)
    if storage == "fp32":
        pos = refb > 0
        assert np.all(out[~pos] == 0)
        assert np.max(np.abs(out[pos] - refb[pos]) / refb[pos]) <= FP32_REL
    else:
        err = np.max(np.abs(out - refb), axis=1) / np.max(np.abs(refb), axis=1)
        assert np.max(err) <= 2 * U16[storage]
    img = lib.apply(torch.from_numpy(Zb[0]).cuda()).cpu().numpy().astype(np.float64)
    big = refb[0] > 1e-6 * refb[0].max()
    tol = FP32_REL if storage == "fp32" else U16[storage] + FP32_REL
    assert np.max(np.abs(img - refb[0])[big] / refb[0][big]) <= tol
    lib.close()
