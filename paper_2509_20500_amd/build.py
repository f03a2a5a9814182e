"""Builds the HIP library ``libdtm.so`` (the method) and ``libdtm_probe.so``
(the benchmark's bandwidth probe) for gfx950, in the package directory.

    python -m paper_2509_20500_amd.build

Every HIP translation unit is compiled with packed-FP32 instructions
disabled (``-packed-fp32-ops``): the compiler then never emits
v_pk_{add,mul,fma}_f32, and float code stays on the scalar-per-lane FP32 path.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdtm.so")
PROBE_LIB = os.path.join(PKG, "libdtm_probe.so")

SOURCES = ["dtm_kernels.hip", "dtm_factored.hip", "dtm_mc.hip", "dtm_mlp.hip", "dtm_host.cpp"]
# the benchmark's bandwidth probe: a library of its own, outside the C-ABI
PROBE_SOURCES = ["dtm_probe.hip"]
HEADERS = ["dtm_internal.h", "dtm_device.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def _build_lib(sources, out, verbose):
    objs = []
    tmp = out + ".tmp"
    for src in sources:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, "-I" + INCLUDE, "-I" + CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        objs.append(obj)
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


def build(verbose: bool = False) -> str:
    """Compile both libraries (always; no staleness check) and return the
    path of the method's library."""
    _build_lib(PROBE_SOURCES, PROBE_LIB, verbose)
    return _build_lib(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
