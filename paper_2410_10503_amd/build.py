"""Builds libmcr.so (the HIP kernels and the C ABI) in the package directory.

    python -m paper_2410_10503_amd.build

hipcc cross-compiles for gfx950 without a GPU being present.
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
LIB = os.path.join(PKG, "libmcr.so")
PROBES_LIB = os.path.join(PKG, "libmcr_probes.so")

SOURCES = ["mcr_api.hip"]
PROBE_SOURCES = ["mcr_probes.hip"]  # roofline probes (measurement only), a library of their own
HEADERS = ["mcr_kernels.h"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep hipcc from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def _compile(sources, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc()] + FLAGS + ["-I", INCLUDE, "-I", CSRC] + [os.path.join(CSRC, s) for s in sources] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile libmcr.so (the HIP kernels and the C ABI) and libmcr_probes.so
    (roofline probes); returns the path of libmcr.so. Always rebuilds."""
    _compile(SOURCES, LIB, verbose)
    _compile(PROBE_SOURCES, PROBES_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
