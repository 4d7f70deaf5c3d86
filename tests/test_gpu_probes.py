"""The measurement probes run through the C ABI, validate their arguments
before any work, and read back plausible rates (a read stream of a 256 MiB
buffer, and matrix-core chains in each format)."""
import pytest

pytestmark = pytest.mark.gpu


def test_probes_run_and_validate():
    import torch
    from paper_2106_09122_amd import psflib
    st = torch.cuda.current_stream().cuda_stream
    sink = torch.zeros(4096, device="cuda")
    buf = torch.zeros(1 << 26, device="cuda")  # 256 MiB
    for slice_ in (False, True):
        for un in (4, 8, 16):
            psflib.probe_hbm_read(buf.data_ptr(), buf.numel() * 4, 2048, un, slice_, sink.data_ptr(), st)
    for kind in (0, 1, 2):
        psflib.probe_mfma(kind, 100, 256, sink.data_ptr(), st)
    torch.cuda.synchronize()
    assert bool((sink == 0).all())  # the sink is written only for an impossible sum
    for args in ((0, 1 << 20, 64, 8, False), (buf.data_ptr(), 1 << 20, 0, 8, False),
                 (buf.data_ptr(), 1 << 20, 64, 5, False), (buf.data_ptr() + 4, 1 << 20, 64, 8, True)):
        with pytest.raises(psflib.PsflibError) as e:
            psflib.probe_hbm_read(*args, sink.data_ptr(), st)
        assert e.value.status == psflib.ERR_INVALID_ARG
    for args in ((3, 10, 64), (1, 0, 64), (1, 10, 0)):
        with pytest.raises(psflib.PsflibError) as e:
            psflib.probe_mfma(*args, sink.data_ptr(), st)
        assert e.value.status == psflib.ERR_INVALID_ARG
