"""Build the HIP library liblsfft.so in-tree for gfx950.

Usage: python -m paper_2009_03762_amd.build [--quick] [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liblsfft.so")
SOURCES = [os.path.join(PKG, "csrc", "lsfft.hip")]
HEADERS = [os.path.join(PKG, "csrc", f) for f in ("fft.hpp", "green.hpp", "kernels.hpp")]
ARCH = os.environ.get("LSFFT_ARCH", "gfx950")


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def command(out=LIB, quick=False):
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           # packed FP32 instructions stay disabled in every HIP build of this library
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", out] + SOURCES
    if quick:
        cmd.insert(1, "-DLSFFT_QUICK_BUILD")
    return cmd


def build(quick=False, verbose=False, out=LIB):
    t0 = time.time()
    tmp = out + ".tmp"
    cmd = command(tmp, quick)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building liblsfft.so")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} in {time.time() - t0:.1f}s", flush=True)
    return out


if __name__ == "__main__":
    build(quick="--quick" in sys.argv, verbose=True)
