"""The planner's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

plan.cpp (host C++, no device code) is compiled with g++ and the sanitizers,
linked with stand-ins for the kernel launchers (tests/host/stubs.cpp) and the
HIP runtime library, and driven by tests/host/host_checks.cpp: Fock-space
arithmetic, host-only plans over many shapes (leaf tilings, inner tables and
descriptors up to m = 255 and m = 24, n = 12), the rank bijection, colex order and
block structure for every m <= 14, n <= 7, option validation and error
paths, and the batch and source planners up to their device check.  Any
sanitizer report, leak or failed check fails the test.  Needs no GPU.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"


def test_planner_host_code_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("needs g++ and the HIP runtime library")
    exe = str(tmp_path / "host_checks")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2204_00602_amd", "csrc"),
           os.path.join(ROOT, "paper_2204_00602_amd", "csrc", "plan.cpp"),
           os.path.join(HERE, "host", "stubs.cpp"), os.path.join(HERE, "host", "host_checks.cpp"),
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    print(res.stdout[-4000:], res.stderr[-4000:])
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    assert "host checks: 0 failure(s)" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
