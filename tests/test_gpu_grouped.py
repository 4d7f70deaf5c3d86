"""Grouped simulation (GPU): scenes of mixed sizes and wavelengths, each with
its own library, as one graph launch; parity with the FP64 oracle per scene."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

U16 = {"bf16": 2.0**-8, "fp16": 2.0**-11}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def work():
    libs, scene_lib, scenes = synth.mixed_workload(B=40, sizes=(16, 24, 32),
                                                   wavelengths=(0.95, 1.0, 1.05, 1.1))
    As = [O.build_library(L["cube"], L["radii"], L["N"], L["S"]) for L in libs]
    refs = [As[L] @ z.astype(np.float64) for L, z in zip(scene_lib, scenes)]
    return libs, scene_lib, scenes, refs


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("autotune", [True, False])
def test_grouped_matches_oracle(torch, work, storage, autotune):
    from paper_2106_09122_amd import psflib
    libs, scene_lib, scenes, refs = work
    L = [psflib.Library(torch.from_numpy(l["cube"]).cuda(), l["radii"], l["N"], l["S"], storage=storage)
         for l in libs]
    Zs = [torch.from_numpy(z).cuda() for z in scenes]
    g = psflib.Grouped(L, scene_lib, Zs, autotune=autotune)
    out = [im.cpu().numpy().astype(np.float64) for im in g.run()]
    torch.cuda.synchronize()
    again = [im.cpu().numpy() for im in g.run()]
    for b, (got, ref) in enumerate(zip(out, refs)):
        assert np.array_equal(got.astype(np.float32), again[b]), "grouped runs must be reproducible"
        if storage == "fp32":
            pos = ref > 0
            assert np.all(got[~pos] == 0)
            assert np.max(np.abs(got[pos] - ref[pos]) / ref[pos]) <= 1e-5, b
        else:
            big = ref > 1e-6 * ref.max()
            assert np.max(np.abs(got - ref)[big] / ref[big]) <= U16[storage] + 1e-5, b
        # the same as a per-scene apply on that library
        single = L[scene_lib[b]].apply(Zs[b]).cpu().numpy().astype(np.float64)
        assert np.max(np.abs(single - got)) <= 2e-5 * np.max(np.abs(got)) + 1e-30
    chunk, ms = g.chunk()
    sh = g.shape()
    assert chunk >= 0 and sh["chunk"] == chunk and sh["rows"] in ((256,) if storage == "fp32" else (64, 128, 256))
    assert (ms > 0) == (autotune and ms > 0)
    g.close()


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_grouped_every_tile_shape(torch, work, storage):
    """Every tile shape the autotuner can pick gives oracle-matching,
    reproducible images: rows per item (16-bit: 256, 128 and 64, the last two
    splitting columns among the workgroup's waves), chunked columns with the
    partials added by the second kernel (chunks of 64 columns: many per
    library, the last one short) and whole columns per item (images written
    directly)."""
    from paper_2106_09122_amd import psflib
    libs, scene_lib, scenes, refs = work
    L = [psflib.Library(torch.from_numpy(l["cube"]).cuda(), l["radii"], l["N"], l["S"], storage=storage)
         for l in libs]
    Zs = [torch.from_numpy(z).cuda() for z in scenes]
    g = psflib.Grouped(L, scene_lib, Zs, autotune=False)
    shapes = [(c, 256) for c in (0, 64, 2048)] if storage == "fp32" else \
             [(c, r) for r in (256, 128, 64) for c in (0, 8, 256)]
    with pytest.raises(RuntimeError):
        g.set_shape(4, 256)  # not a whole number of blocks
    with pytest.raises(RuntimeError):
        g.set_shape(0, 32)
    for chunk, rows in shapes:
        g.set_shape(chunk, rows)
        assert g.shape()["chunk"] == chunk and g.shape()["rows"] == rows
        out = [im.cpu().numpy().astype(np.float64) for im in g.run()]
        again = [im.cpu().numpy() for im in g.run()]
        for b, (got, ref) in enumerate(zip(out, refs)):
            assert np.array_equal(got.astype(np.float32), again[b]), (chunk, rows, b)
            if storage == "fp32":
                pos = ref > 0
                assert np.all(got[~pos] == 0)
                assert np.max(np.abs(got[pos] - ref[pos]) / ref[pos]) <= 1e-5, (chunk, rows, b)
            else:
                big = ref > 1e-6 * ref.max()
                assert np.max(np.abs(got - ref)[big] / ref[big]) <= U16[storage] + 1e-5, (chunk, rows, b)
    g.close()


def test_grouped_empty_and_unused_libraries(torch, work):
    from paper_2106_09122_amd import psflib
    libs = work[0]
    L = [psflib.Library(torch.from_numpy(l["cube"]).cuda(), l["radii"], l["N"], l["S"]) for l in libs[:3]]
    g = psflib.Grouped(L, [], [], autotune=True)
    assert g.run() == []
    z = torch.from_numpy(work[2][0]).cuda() if work[1][0] < 3 else None
    if z is not None:
        g2 = psflib.Grouped(L, [work[1][0]], [z])  # two of three libraries unused
        ref = work[3][0]
        got = g2.run()[0].cpu().numpy().astype(np.float64)
        pos = ref > 0
        assert np.max(np.abs(got[pos] - ref[pos]) / ref[pos]) <= 1e-5


@pytest.fixture(scope="module")
def crowded():
    """Two libraries with odd pixel counts (15^2, 17^2: the unaligned load path)
    and about 20 scenes each, so each library takes a full and a partial scene
    group."""
    libs, scene_lib, scenes = synth.mixed_workload(B=40, sizes=(15, 17), wavelengths=(1.0,))
    As = [O.build_library(L["cube"], L["radii"], L["N"], L["S"]) for L in libs]
    refs = [As[L] @ z.astype(np.float64) for L, z in zip(scene_lib, scenes)]
    return libs, scene_lib, scenes, refs


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_grouped_crowded_odd_sizes(torch, crowded, storage):
    from paper_2106_09122_amd import psflib
    libs, scene_lib, scenes, refs = crowded
    assert max(np.bincount(scene_lib)) > 16
    L = [psflib.Library(torch.from_numpy(l["cube"]).cuda(), l["radii"], l["N"], l["S"], storage=storage)
         for l in libs]
    Zs = [torch.from_numpy(z).cuda() for z in scenes]
    g = psflib.Grouped(L, scene_lib, Zs, autotune=True)
    out = [im.cpu().numpy().astype(np.float64) for im in g.run()]
    for b, (got, ref) in enumerate(zip(out, refs)):
        if storage == "fp32":
            pos = ref > 0
            assert np.all(got[~pos] == 0)
            assert np.max(np.abs(got[pos] - ref[pos]) / ref[pos]) <= 1e-5, b
        else:
            big = ref > 1e-6 * ref.max()
            assert np.max(np.abs(got - ref)[big] / ref[big]) <= U16[storage] + 1e-5, b
    g.close()


@pytest.fixture(scope="module")
def full():
    """The mixed workload at its full size (sizes 64, 96, 128 x 11 wavelengths:
    33 libraries, 256 scenes), each scene replaced by one supported on 8 seeded
    columns of its library, so the oracle builds only the columns each image
    needs; the plan and launch are those of the full workload."""
    libs, scene_lib, _ = synth.mixed_workload()
    rng = np.random.default_rng(77)
    scenes, refs = [], []
    for L in scene_lib:
        lib = libs[L]
        ncols = lib["N"] ** 2
        cols = np.sort(rng.choice(ncols, 8, replace=False))
        z = np.zeros(ncols, dtype=np.float32)
        z[cols] = (rng.random(8) * 10.0 ** rng.uniform(-9, -7, 8)).astype(np.float32)
        A = O.build_library(lib["cube"], lib["radii"], lib["N"], lib["S"], columns=cols)
        scenes.append(z)
        refs.append(A @ z[cols].astype(np.float64))
    return libs, scene_lib, scenes, refs


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_grouped_full_workload_sampled(torch, full, storage):
    from paper_2106_09122_amd import psflib
    libs, scene_lib, scenes, refs = full
    assert len(libs) == 33 and len(scene_lib) == 256
    L = [psflib.Library(torch.from_numpy(l["cube"]).cuda(), l["radii"], l["N"], l["S"], storage=storage)
         for l in libs]
    Zs = [torch.from_numpy(z).cuda() for z in scenes]
    g = psflib.Grouped(L, scene_lib, Zs, autotune=True)
    out = [im.cpu().numpy().astype(np.float64) for im in g.run()]
    for b, (got, ref) in enumerate(zip(out, refs)):
        if storage == "fp32":
            pos = ref > 0
            assert np.all(got[~pos] == 0)
            assert np.max(np.abs(got[pos] - ref[pos]) / ref[pos]) <= 1e-5, b
        else:
            big = ref > 1e-6 * ref.max()
            assert np.max(np.abs(got - ref)[big] / ref[big]) <= U16[storage] + 1e-5, b
    g.close()
    for lib in L:
        lib.close()
