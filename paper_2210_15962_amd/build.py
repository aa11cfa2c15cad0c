"""Build liblabs.so in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2210_15962_amd.build`` (or ``build()`` from Python).
The shared library lands next to this file; the Python binding loads it from
there.  Set ``LABS_SAVE_TEMPS=1`` to keep the gfx950 assembly for inspection.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblabs.so")
ARCH = "gfx950"

# Packed FP32 VALU ops are switched off for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    extra = []
    if os.environ.get("LABS_SAVE_TEMPS"):
        extra = ["-save-temps=obj"]
    # The device translation units compile in parallel (the walk kernels take minutes).
    procs = []
    for src in ("labs_kernels.hip", "labs_full.hip", "labs_full_serve.hip", "labs_noalloc.hip"):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc, "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS, *extra, "-c",
               os.path.join(CSRC, src), "-o", obj]
        print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for proc, cmd in procs:
        if proc.wait() != 0:
            raise subprocess.CalledProcessError(proc.returncode, cmd)
    for host_src in ("labs_api.cpp", "labs_serve.cpp", "labs_solve.cpp"):
        obj = os.path.join(bdir, host_src.replace(".cpp", ".o"))
        _run([hipcc, *COMMON, "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(CSRC, host_src),
              "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-pthread", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
