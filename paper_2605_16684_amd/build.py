"""Build step for the HIP library libesdg.so (gfx950 only).

hipcc compiles csrc/esdg_api.hip (which includes the device code) into a
shared library beside this file.  Packed FP32 instructions are disabled
(-packed-fp32-ops); no fast-math.  The library carries a hash of the
sources it was built from (esdg_version()), and the Python binding refuses
to load a library whose hash differs from the sources in the tree.
"""
import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "esdg_api.hip")
LIB = os.path.join(HERE, "libesdg.so")
ARCH = "gfx950"


def sources():
    """Every file the library is compiled from: the HIP sources and headers
    under csrc/ and the public header."""
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                   glob.glob(os.path.join(HERE, "csrc", "*.hpp")))
    return files + [os.path.join(ROOT, "include", "esdg.h")]


DEPS = sources()


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) over the names and bytes of sources()."""
    h = hashlib.sha256()
    for f in sources():
        h.update(os.path.relpath(f, ROOT).encode())
        h.update(b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def hipcc_cmd(out, extra=()):
    return ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-ffp-contract=fast-honor-pragmas", "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
            f'-DESDG_SOURCE_HASH="{source_hash()}"', *extra, "-o", out, SRC]


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
    return any(os.path.getmtime(d) > t for d in sources())


if __name__ == "__main__":
    print(build(verbose=True))
