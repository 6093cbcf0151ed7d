"""The library's host code (offsets, workspace layout, index tables, argument
checks) built with AddressSanitizer and UndefinedBehaviorSanitizer on the
host pass only and run on the CPU (tests/native/host_checks.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    # the program launches no kernel: only the smallest size's kernels are
    # compiled (PTYCHO_KERNEL_N_MAX), the host code is the library's own
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-DPTYCHO_KERNEL_N_MAX=8",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2008_11511_amd", "csrc"),
           os.path.join(ROOT, "paper_2008_11511_amd", "csrc", "ptycho.hip"),
           os.path.join(ROOT, "paper_2008_11511_amd", "csrc", "inst_8.hip"),
           os.path.join(ROOT, "tests", "native", "host_checks.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks: 0 failures" in r.stdout
