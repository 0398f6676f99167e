"""Build libmpr.so (the C-ABI library and its gfx950 kernels) in place.

    python -m paper_1710_03038_amd.build

Compiles every source under csrc/ with hipcc for gfx950 only.  Packed FP32
instructions are disabled (-packed-fp32-ops): the kernels are written as
scalar float code and must not be turned into v_pk_* forms.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpr.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "api.hip")]


def hipcc_command(out=LIB, extra=()):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *extra, *SOURCES, "-o", out]


def build(verbose=True):
    """Compile libmpr.so next to this file; raise on failure."""
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmpr.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
