"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/sanitize/host_driver.cpp drives descriptor validation, workspace layout, the CG chunk
policy and the argument checks of the entry points.  It is linked with the library's own host
driver and launch geometry, compiled as host C++ (no device code, so no GPU is needed; the kernel
launchers are host stand-ins that no call reaches) with both sanitizers on and errors fatal.
"""

import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_03804_amd", "csrc")


def clangxx():
    for c in (os.environ.get("HIP_CLANGXX"), "/opt/rocm/lib/llvm/bin/clang++"):
        if c and os.path.exists(c):
            return c
    return shutil.which("clang++")


@pytest.mark.slow
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    cc = clangxx()
    if cc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("ROCm clang++ and HIP headers not available")
    tmp = tempfile.mkdtemp(prefix="fh_sanitize_")
    try:
        # the host driver is HIP source without device code: compiled as host C++ from a copy
        drv = os.path.join(tmp, "fft_homog_host.cpp")
        shutil.copy(os.path.join(CSRC, "fft_homog.hip"), drv)
        exe = os.path.join(tmp, "host_driver")
        cmd = [cc, "-x", "c++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
               drv, os.path.join(CSRC, "launch_geometry.cpp"), os.path.join(ROOT, "tests", "sanitize", "launch_stubs.cpp"),
               os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
               "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
        assert "0 failures" in out
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
