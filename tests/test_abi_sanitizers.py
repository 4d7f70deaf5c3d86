"""The C ABI's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: the sanitizer flags go through
-Xarch_host, the gfx950 device code is compiled as usual), driven by
tests/abi_sanitize.c through every argument check and error path.  The driver
makes no call that could reach a device, so this runs without a GPU."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests.conftest import ROOT

SAN = ["address", "undefined"]


def _host_san_flags():
    out = []
    for s in SAN:
        out += ["-Xarch_host", f"-fsanitize={s}"]
    return out + ["-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_abi_host_code_is_sanitizer_clean(tmp_path):
    from paper_2106_09122_amd import _build
    hipcc = _build.hipcc()
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang not found")
    flags = [f for f in _build.compile_flags() if f != "-O3"] + ["-O1", "-g"] + _host_san_flags()

    def one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(_build.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(one, _build.SOURCES))
    drv = str(tmp_path / "abi_sanitize.o")
    sanitize = "-fsanitize=" + ",".join(SAN)
    r = subprocess.run([clang, "-O1", "-g", sanitize, "-fno-sanitize-recover=all",
                        "-I", os.path.join(ROOT, "include"), "-c",
                        os.path.join(ROOT, "tests", "abi_sanitize.c"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "abi_sanitize")
    r = subprocess.run([clang + "++", sanitize, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-Wl,-rpath,/opt/rocm/lib", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    supp = tmp_path / "lsan.supp"
    # allocations the HIP/HSA runtimes keep for the process are theirs, not leaks of this code
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler-register\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={supp}"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "abi_sanitize ok" in r.stdout
