"""Build the HIP library in place: hipcc for gfx950 -> libsphere_poisson.so
next to this file.  Each translation unit compiles to an object of its own,
in parallel, and the objects link into the shared library.  Run as
``python -m paper_1510_08094_amd.build``."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# the solver's host code and small kernels, the kernel builds of its passes (one unit per group),
# and the Gaussian-elimination constructor
SRCS = [os.path.join(CSRC, name) for name in (
    "sphere_poisson.hip", "sp_inst_solve.hip", "sp_inst_mixed_small.hip", "sp_inst_mixed_large.hip",
    "sp_inst_mixed_fixed.hip", "sp_inst_mixed_pick.hip", "sp_inst_batch_lambda.hip", "sp_inst_batch_theta64.hip",
    "sp_inst_batch_theta_first.hip", "sp_inst_batch_theta_resid.hip", "sp_ge.hip")]
OUT = os.path.join(HERE, "libsphere_poisson.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
            # packed FP32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: %s" % " ".join(cmd))


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the CPU checks
# of the C ABI (argument validation, plan and batch-plan bookkeeping): each
# -fsanitize applies to the host compilation only; the device code is built as
# usual.  The result is a separate library that only CPU tests load (with the
# sanitizer runtime preloaded, see README).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
OUT_SANITIZE = os.path.join(OBJDIR, "libsphere_poisson_asan.so")


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    objdir = os.path.join(OBJDIR, "asan") if sanitize else OBJDIR
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s)[:-4] + ".o") for s in SRCS]
    cc = hipcc()
    extra = SANITIZE if sanitize else []
    jobs = jobs or min(len(SRCS), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, [cc] + flags() + extra + ["-c", s, "-o", o], verbose)
                  for s, o in zip(SRCS, objs)]:
            f.result()
    out = OUT_SANITIZE if sanitize else OUT
    tmp = out + ".tmp%d" % os.getpid()
    _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + extra + ["-o", tmp] + objs, verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
