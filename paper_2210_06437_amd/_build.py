"""Build liboctohydro.so in-tree with hipcc for gfx950.

The library's translation units (host code and small kernels; the fused
substep in binary64 and in binary32 storage; the 3D step, its instantiations
spread over eight units; the table builder) are compiled to objects in
parallel and linked into one shared library.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liboctohydro.so")
# every translation unit of the library (the 3D step's instantiations are
# spread over several units so that they compile in parallel)
SOURCES = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [os.path.join(CSRC, "table.cpp")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# binary64 results must be reproducible operation by operation: no FMA
# contraction, IEEE division and square root; packed FP32 instructions are
# disabled for all device code.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]
# hipcc's host pass warns that it does not know the packed-fp32 feature
_NOISE = "is not a recognized feature for this target"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if _NOISE not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    objdir = tempfile.mkdtemp(prefix="octohydro_obj_")
    try:
        objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in SOURCES]
        with ThreadPoolExecutor(len(SOURCES)) as ex:
            list(ex.map(lambda so: _run([HIPCC, *FLAGS, *extra, "-c", "-o", so[1], so[0]],
                                        verbose), zip(SOURCES, objs)))
        tmp = out + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
