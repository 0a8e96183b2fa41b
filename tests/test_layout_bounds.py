"""Host-side bounds check of the decode kernel's LDS layout over every launch
shape the host can choose (tests/sanitize/layout_main.cpp), built with
AddressSanitizer and UBSan.  No GPU is needed."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"
CSRC = os.path.join(ROOT, "paper_2405_01808_amd", "csrc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_lds_layout_regions_in_bounds(tmp_path):
    exe = str(tmp_path / "layout_check")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(HERE, "sanitize", "layout_main.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert run.returncode == 0, run.stdout[-3000:] + run.stderr[-3000:]
    assert " 0 failures" in run.stdout
