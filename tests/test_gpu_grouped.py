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
    assert chunk > 0 and (ms > 0) == (autotune and ms > 0)
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
