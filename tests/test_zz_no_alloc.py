"""The allocation-free apply (psflib_apply_noalloc), through the C ABI,
against psflib_apply: the same kernels and summation order with the partial
sums in the library's fixed device array instead of pool memory, so the
images must be bitwise equal.  Two calls in a row on one GPU, the second on a
smaller library (fewer partials than the first left in the array), in each
storage form."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_noalloc_apply_equals_apply(storage):
    import torch
    from paper_2106_09122_amd import psflib
    st = torch.cuda.current_stream().cuda_stream
    # 128^2 (32 x 16384 partial sums in FP32), then 32^2 (64 x 1024)
    for d in (synth.config_inputs(2), synth.config_inputs(1)):
        print(f"noalloc {storage}: n={d['n']} N={d['N']}", flush=True)
        lib = psflib.Library(torch.from_numpy(d["cube"]).cuda(), d["radii"], d["N"], d["S"],
                             storage=storage)
        scenes = [torch.from_numpy(d["scene"]).cuda(),
                  torch.from_numpy(np.random.default_rng(d["n"]).random(d["N"] ** 2)
                                   .astype(np.float32)).cuda()]
        for Z in scenes:
            ref = torch.empty(lib.M, device="cuda")
            out = torch.full((lib.M,), float("nan"), device="cuda")
            psflib.apply(lib.h, Z.data_ptr(), ref.data_ptr(), st)
            psflib.apply_noalloc(lib.h, Z.data_ptr(), out.data_ptr(), st)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
        lib.close()


def test_noalloc_rejects_bad_arguments_before_any_work():
    import torch
    from paper_2106_09122_amd import psflib
    d = synth.config_inputs(1)
    lib = psflib.Library(torch.from_numpy(d["cube"]).cuda(), d["radii"], d["N"], d["S"])
    st = torch.cuda.current_stream().cuda_stream
    Z = torch.from_numpy(d["scene"]).cuda()
    out = torch.full((lib.M + 4,), 7.0, device="cuda")
    for args in ((0, Z.data_ptr(), out.data_ptr()), (lib.h, 0, out.data_ptr()),
                 (lib.h, Z.data_ptr(), out.data_ptr() + 4)):
        with pytest.raises(psflib.PsflibError) as e:
            psflib.apply_noalloc(*args, st)
        assert e.value.status == psflib.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    lib.close()
