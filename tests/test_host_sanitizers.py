"""The library's host C++ (octree meshing, hanging-node constraints, prolongation, dense
coarsest inverse) built with AddressSanitizer and UndefinedBehaviorSanitizer by the host
compiler and run on the CPU (tests/native/octree_host_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_octree_code_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    csrc = os.path.join(ROOT, "paper_1408_6497_amd", "csrc")
    exe = str(tmp_path / "octree_host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", csrc, "-I", "/opt/rocm/include",
           os.path.join(csrc, "gmg_octree_host.cpp"), os.path.join(csrc, "gmg_setup_math.cpp"),
           os.path.join(ROOT, "tests", "native", "octree_host_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    print(run.stdout, run.stderr)
    assert run.returncode == 0, run.stderr[-2000:]
    assert "q=2:" in run.stdout
