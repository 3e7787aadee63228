"""Build the in-tree shared library ``libamg.so`` for gfx950.

The host setup (plain C++) is compiled with the system C++ compiler; the HIP
sources with hipcc for gfx950; the library links rocSOLVER/rocBLAS (dense LU
of the coarsest level at setup time only).  Run ``python -m
paper_1811_05704_amd.build`` or call :func:`build`.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libamg.so")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SOURCES = ["host_setup.cpp", "block_setup.cpp", "field_split.cpp"]
HIP_SOURCES = ["solver.hip", "serve.hip", "galerkin.hip", "noalloc.hip", "staging.hip"]

# Host arithmetic of the setup follows each definition's natural order with
# separate multiply and add (no contraction), for reproducible hierarchies.
CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra", "-pthread",
            "-I" + os.path.join(ROCM, "include")]
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROCM, "include"), "-Wall",
]
LDFLAGS = ["-shared", "-L" + os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas", "-lrocprofiler-sdk-roctx",
           "-pthread",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in proc.stdout.splitlines() if "packed-fp32-ops" not in l)
    if proc.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, ["g++", *CXXFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]))
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, [HIPCC, *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]))
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, cmd) for _, cmd in jobs]:
            f.result()
    objs = [obj for obj, _ in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", *objs, *LDFLAGS, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
