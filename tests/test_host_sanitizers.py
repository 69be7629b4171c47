"""The library's host sources (CSR -> CSRC split, plans, colouring, batch
plans, features, selector inference) built with g++ under AddressSanitizer
and UndefinedBehaviorSanitizer and driven by tests/host_sanitize.cpp on
seeded random patterns and edge cases.  No GPU: the driver stubs the three
HIP runtime calls the host code references."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1003_0952_amd", "csrc")
HOST_SOURCES = ["csrc_host.cpp", "csrc_plan.cpp", "csrc_batch.cpp", "csrc_mlp_host.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_sources_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
            "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{os.path.join(ROOT, 'include')}",
            "-o", exe, os.path.join(ROOT, "tests", "host_sanitize.cpp")]
           + [os.path.join(CSRC, s) for s in HOST_SOURCES])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "sanitize ok" in r.stdout, (r.stdout[-2000:], r.stderr[-6000:])
