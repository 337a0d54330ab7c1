"""The library's host code under AddressSanitizer (host side only; device code
is built as usual): a test program linked with the library sources checks the input
validation of pdlpb_create, every entry point with a NULL context and, on a
machine without a GPU, the failure path of a well-formed create.  Any memory
error or leak in that code fails the program's exit status.  The same program
with --device runs a context through every entry point on a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_21990_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_abi_host_code_under_address_sanitizer(tmp_path):
    exe = tmp_path / "abi_check"
    cmd = [HIPCC, "-O1", "-g", "--offload-arch=gfx950", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           "-fno-gpu-rdc", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-x", "hip",
           os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "pdlpb.cpp"),
           os.path.join(ROOT, "tests", "asan", "abi_check.cpp"), "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-3000:]
    # allocations the ROCm runtime keeps until exit are not the library's
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libhsa-runtime64\nleak:libamdhip64\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", LSAN_OPTIONS=f"suppressions={supp}")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "ok (0 failures)" in r.stdout, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
