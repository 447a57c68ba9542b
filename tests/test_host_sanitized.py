"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

fpw_host.cpp is compiled with g++ together with CPU stand-ins for the HIP calls
it makes (tests/c/hip_stub.cpp: device memory is host memory, kernel launches
do nothing) and a driver (tests/c/host_driver.cpp) that creates, evaluates and
destroys every kind of plan and launch shape and calls every other entry
point.  Any out-of-bounds access, use after free, leak or undefined behaviour
in the plan, shape, queue, graph-cache or autotune logic stops the program;
the driver also checks each call's status.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_host_runtime_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path / "host_check")
    sanitize = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    cmd = [gxx, "-std=c++17", "-g", "-O1", *sanitize, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2502_00243_amd", "csrc"),
           os.path.join(ROOT, "paper_2502_00243_amd", "csrc", "fpw_host.cpp"), os.path.join(HERE, "c", "hip_stub.cpp"),
           os.path.join(HERE, "c", "host_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path / "tune_cache.txt")], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "failures: 0" in r.stdout
    # the autotune run wrote its cache, and the second plan found it
    assert (tmp_path / "tune_cache.txt").read_text().startswith("gfx")
