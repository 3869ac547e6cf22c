"""The library's host-side C++ (reference tables, quadrature, local-matrix and
diagonal tables, the C0 maps) built with AddressSanitizer and
UndefinedBehaviorSanitizer by the host compiler and run on a driver that
exercises every builder and both maps with their error paths
(tests/host_sanitize_driver.cpp).  No device code is compiled."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_04644_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs the host compiler and the HIP headers")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    srcs = [os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), os.path.join(CSRC, "shp_tables.cpp"),
            os.path.join(CSRC, "shp_c0.cpp")]
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I" + os.path.join(ROOT, "include")]
    r = subprocess.run(["g++"] + flags + srcs + ["-o", exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ok: 0 failures" in r.stdout, (r.stdout[-4000:], r.stderr[-4000:])
