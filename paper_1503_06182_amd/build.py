"""Build the gfx950 HIP library in-tree: paper_1503_06182_amd/libvegas.so.

hipcc cross-compiles for gfx950 without a GPU.  Packed-FP32 instructions are
disabled for device code (-packed-fp32-ops); contraction is left on for the
physics and switched off by pragma where a step must round as written.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libvegas.so")
SOURCES = [os.path.join(HERE, "csrc", "vegas.hip"), os.path.join(HERE, "csrc", "flow.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("device_common.hpp", "integrands.hpp", "adjoint.hpp", "flow.hpp")] + [
    os.path.join(ROOT, "include", "vegas.h")]
ARCH = os.environ.get("VEGAS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
