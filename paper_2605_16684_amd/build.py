"""Build step for the HIP library libesdg.so (gfx950 only).

hipcc compiles csrc/esdg_api.hip (which includes the device code) into a
shared library beside this file.  Packed FP32 instructions are disabled
(-packed-fp32-ops); no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "esdg_api.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "esdg_device.hpp"), os.path.join(HERE, "csrc", "esdg_mixed.hpp"),
        os.path.join(ROOT, "include", "esdg.h")]
LIB = os.path.join(HERE, "libesdg.so")
ARCH = "gfx950"


def hipcc_cmd(out, extra=()):
    return ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-ffp-contract=fast-honor-pragmas", "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
            *extra, "-o", out, SRC]


def build(verbose: bool = False, extra=()) -> str:
    cmd = hipcc_cmd(LIB + ".tmp", extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
