"""The library's host code under AddressSanitizer (CPU only): the HIP sources
and tests/asan_host_abi.cpp are built with the sanitizer on the host
compilation only (device code is compiled as usual and never run), then the
driver exercises every host-only routine and the argument validation of the
device entry points on exact-size heap buffers."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not installed")
def test_host_code_is_clean_under_address_sanitizer(tmp_path):
    from paper_2503_05168_amd.build import sources
    exe = tmp_path / "asan_host_abi"
    cmd = [CLANG, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-ffp-contract=off", "-munsafe-fp-atomics",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2503_05168_amd", "csrc"),
           *sources(), "-x", "c++", os.path.join(ROOT, "tests", "asan_host_abi.cpp"),
           "--hip-link", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "0 failed checks" in r.stdout
    shutil.rmtree(tmp_path, ignore_errors=True)
