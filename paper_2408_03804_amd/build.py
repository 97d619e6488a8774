"""Build the HIP shared library libfft_homog.so for gfx950 (in-tree).

Usage:  python -m paper_2408_03804_amd.build   (or call build()).
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfft_homog.so")
SOURCES = ["kernels.hip", "kernels_chirp.hip", "kernels_fixed.hip", "fft_homog.hip", "cnn.hip", "launch_geometry.cpp", "noalloc_scratch.hip"]
HEADERS = ["common.h", "dual.h", "materials.h", "fft_lds.h", "kernels.h", "pass_kernels.h"]

FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
# The CG kernels' dual numbers are seeded with literal zeros (one-hot partials); with these two
# flags the compiler may drop products with them and additions of them, which is exact for
# finite values (results change at most in the sign of a zero) and removes a sixth of the
# forward x pass's time.  They also let the compiler assume no NaN or Inf, so every domain and
# breakdown test in those kernels is an integer test on the exponent bits (finite_bits).
PER_FILE = {"kernels.hip": ["-ffinite-math-only", "-fno-signed-zeros"],
            "kernels_chirp.hip": ["-ffinite-math-only", "-fno-signed-zeros"],
            "kernels_fixed.hip": ["-ffinite-math-only", "-fno-signed-zeros"]}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose=False, extra_flags=()):
    """Compile every source (in parallel) and link libfft_homog.so (always recompiles)."""
    import tempfile

    tmp = tempfile.mkdtemp(prefix="fft_homog_build_")
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + FLAGS + PER_FILE.get(src, []) + list(extra_flags) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed = True
    if failed:
        raise RuntimeError("hipcc failed building libfft_homog.so")
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libfft_homog.so")
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmp)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
