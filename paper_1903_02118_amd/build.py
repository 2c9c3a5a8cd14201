"""Build of the HIP library `libbie.so` for gfx950 (in-tree).

Compiles the device code (kernels.hip, probe.hip, aca.hip) and the host code (api.cpp,
fdph_setup.cpp) with hipcc and links one shared library next to this file.
Run `python -m paper_1903_02118_amd.build` or call `build()`.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbie.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall", "-Wno-unused-function"]
# Device code: packed-FP32 instructions disabled (the compiler emits scalar FP32
# operations instead of v_pk_* forms).
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-fopenmp"]

SOURCES = [
    ("kernels.hip", DEVICE),
    ("probe.hip", DEVICE),
    ("aca.hip", DEVICE),
    ("api.cpp", HOST),
    ("fdph_setup.cpp", HOST),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libbie.so; returns its path."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at " + HIPCC)
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        _run([HIPCC, *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fopenmp", "-o", tmp, *objs], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
