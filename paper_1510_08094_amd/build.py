"""Build the HIP library in place: hipcc for gfx950 -> libsphere_poisson.so
next to this file.  Run as ``python -m paper_1510_08094_amd.build``."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# the solver, and the Gaussian-elimination constructor in a translation unit of its own
SRCS = [os.path.join(HERE, "csrc", "sphere_poisson.hip"), os.path.join(HERE, "csrc", "sp_ge.hip")]
OUT = os.path.join(HERE, "libsphere_poisson.so")
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-shared",
            # packed FP32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + flags() + ["-o", tmp] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for %s" % " ".join(SRCS))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
