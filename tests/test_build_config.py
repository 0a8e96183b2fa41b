"""The library's build description: per-file device flags name real sources,
and the kernel hash that keys the committed profiles covers the kernel's
files and its build flags.  No GPU and no compiler needed."""
import os

from paper_2405_01808_amd import build


def test_flagged_files_are_sources():
    for f in build.FILE_FLAGS:
        assert f in build.SOURCES


def test_sources_and_kernel_files_exist():
    for f in build.SOURCES + build.KERNEL_FILES:
        assert os.path.isfile(os.path.join(build.CSRC, f)), f


def test_compile_command_carries_the_file_flags():
    for f in build.SOURCES:
        cmd = build.compile_command(f, "x.o")
        flags = build.FILE_FLAGS.get(f, [])
        if flags:
            i = cmd.index(flags[0])
            assert cmd[i:i + len(flags)] == flags
        # every file keeps packed FP32 instructions out of its code
        assert "-packed-fp32-ops" in cmd


def test_kernel_hash_covers_the_build_flags(monkeypatch):
    before = build.kernel_source_sha256()
    assert before == build.kernel_source_sha256()
    flags = {k: list(v) for k, v in build.FILE_FLAGS.items()}
    flags["grand_kernels_n128.hip"] = flags.get("grand_kernels_n128.hip", []) + ["-O2"]
    monkeypatch.setattr(build, "FILE_FLAGS", flags)
    assert build.kernel_source_sha256() != before
