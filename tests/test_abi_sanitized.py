"""The C ABI's host code built with AddressSanitizer and UBSan (host side
only; device code is compiled normally) and driven through its validation
and error paths (tests/sanitize/abi_main.cpp).  No GPU is needed."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"
CSRC = os.path.join(ROOT, "paper_2405_01808_amd", "csrc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_paths_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "abi_asan")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    from paper_2405_01808_amd.build import SOURCES   # every source of the library
    cmd += [os.path.join(CSRC, f) for f in SOURCES]
    cmd += [os.path.join(HERE, "sanitize", "abi_main.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert build.returncode == 0, build.stderr[-3000:]
    # the HIP runtime keeps allocations for the process lifetime: no leak check
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr[-3000:]
    assert "runtime error" not in run.stderr, run.stderr[-3000:]
    assert "0 failures" in run.stdout
