"""Static check of the 16-bit GEMM's memory pipeline in the compiled gfx950
code.  Its ring-slot wait ('at most 2 (4 + C) vector-memory operations
outstanding' before each stage barrier, C = 2 LDS copies per lane and stage
for the 128-scene tile, 4 for the 256-scene tile) is only correct if,
between two stage barriers, each lane issues exactly 4 library loads to
registers and C buffer-to-LDS copies, nothing else that counts against
vmcnt (no stores, no scratch spills), and no such operation sits between a
loop header and its first barrier.  The device assembly is compiled here
from the source with the library's own flags and parsed."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from tests.conftest import ROOT

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")

VMEM = re.compile(r"^\s*(global|buffer|flat|scratch)_\w+")


@pytest.fixture(scope="module")
def asm():
    from paper_2106_09122_amd import _build
    flags = [f for f in _build.compile_flags() if f not in ("-fPIC",)]
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "gemm.s")
        subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S",
                        os.path.join(ROOT, "paper_2106_09122_amd", "csrc", "gemm.hip"), "-o", out],
                       check=True, capture_output=True)
        return open(out).read()


def kernel_bodies(text):
    """(name, library loads to registers, LDS copies) per stage of every
    16-bit GEMM kernel: the 4-wave kernels load 4 library fragments and copy
    TN/64 scene fragments per lane; the 8-wave kernel copies 2 library and 2
    scene fragments per lane into LDS."""
    names = re.findall(r"^(_ZN6psflib15gemm_h16_kernel\w+):", text, re.M)
    assert len(names) == 8  # bf16 and fp16, 128- and 256-scene tiles, with and without the NT hint
    for name in names:
        tn = int(re.search(r"ILb[01]ELi(\d+)E", name).group(1))
        body = text[text.index(name + ":"):]
        yield name, 4, tn // 64, body[:body.index("s_endpgm")].splitlines()
    w8 = re.findall(r"^(_ZN6psflib18gemm_h16_w8_kernel\w+):", text, re.M)
    assert len(w8) == 2  # bf16 and fp16
    for name in w8:
        body = text[text.index(name + ":"):]
        yield name, 0, 4, body[:body.index("s_endpgm")].splitlines()


def test_stage_issue_pattern(asm):
    for name, reg_loads, copies_per_stage, lines in kernel_bodies(asm):
        assert not any("scratch_" in l for l in lines), name
        # a stage barrier: the ring wait then s_barrier
        wait = f"s_waitcnt vmcnt({2 * (reg_loads + copies_per_stage)})"
        bars = [i for i, l in enumerate(lines)
                if "s_barrier" in l and i > 0 and wait in lines[i - 1]]
        assert len(bars) >= 8, name
        for a, b in zip(bars, bars[1:]):
            seg = lines[a:b]
            loads = sum("global_load_dwordx4" in l for l in seg)
            copies = sum(re.search(r"buffer_load_dwordx4\b.*\blds\b", l) is not None for l in seg)
            other = [l for l in seg if VMEM.match(l) and "global_load_dwordx4" not in l
                     and not re.search(r"buffer_load_dwordx4\b.*\blds\b", l)]
            assert (loads, copies) == (reg_loads, copies_per_stage) and not other, (name, a, loads, copies, other)
        # loop headers: nothing counted against vmcnt before the first barrier
        for i, l in enumerate(lines):
            if "Loop Header" in l:
                nxt = [b for b in bars if b > i]
                if nxt:
                    assert not any(VMEM.match(x) for x in lines[i:nxt[0]]), (name, i)
