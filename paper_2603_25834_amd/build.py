"""Build step of the gfx950 library ``libaslam.so`` (hipcc, in-tree).

Every HIP source is compiled for gfx950 with FP contraction off (the pose and
covariance arithmetic is specified operation by operation), correctly rounded
FP32 division, and packed-FP32 instructions disabled; each to an object of its
own (the sources in parallel), then linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libaslam.so")

SOURCES = ["capi.hip", "env_kernels.hip", "policy_capi.hip", "slam.hip", "fixedlag.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_library(verbose: bool = False) -> str:
    """Each source compiled to an object (in parallel), then linked."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="aslam_build_") as work:
        jobs = []
        for src in sources():
            obj = os.path.join(work, os.path.basename(src) + ".o")
            jobs.append(([hipcc()] + HIPCC_FLAGS + inc + ["-c", src, "-o", obj], obj))
        if verbose:
            for cmd, _ in jobs:
                print(" ".join(cmd), flush=True)
        with ThreadPoolExecutor(max_workers=min(len(jobs), max(1, os.cpu_count() or 1))) as ex:
            for f in [ex.submit(subprocess.check_call, cmd) for cmd, _ in jobs]:
                f.result()
        tmp = LIB + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o in jobs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
