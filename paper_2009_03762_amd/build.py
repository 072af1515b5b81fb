"""Build the HIP library liblsfft.so in-tree for gfx950.

The host side, the FP32 and FP64 pass kernels (x side; y, z and strain x)
and the 1D solver are six translation units, compiled in parallel and linked
into one shared library.

Usage: python -m paper_2009_03762_amd.build [--quick] [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liblsfft.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("lsfft.hip", "launch_f32.hip", "launch_f32_yz.hip", "launch_f64.hip",
                                                  "launch_f64_yz.hip", "solve1d.hip")]
HEADERS = [os.path.join(PKG, "csrc", f) for f in ("fft.hpp", "green.hpp", "kernels.hpp", "disp.hpp", "reduce.hpp",
                                                  "solver.hpp", "launch.hpp")]
ARCH = os.environ.get("LSFFT_ARCH", "gfx950")


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags(quick=False, extra=()):
    flags = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             # packed FP32 instructions stay disabled in every HIP build of this library
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]
    if quick:
        flags.append("-DLSFFT_QUICK_BUILD")
    return flags + list(extra)


def commands(objdir, out=LIB, quick=False, extra=()):
    """(compile commands, one per source; the link command).  `extra`: further
    compiler flags for every unit (e.g. -D overrides of the tile constants)."""
    objs = [os.path.join(objdir, os.path.splitext(os.path.basename(s))[0] + ".o") for s in SOURCES]
    comp = [compile_flags(quick, extra) + ["-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs
    return comp, link


def build(quick=False, verbose=False, out=LIB, extra=()):
    t0 = time.time()
    tmp = out + ".tmp"
    with tempfile.TemporaryDirectory(prefix="lsfft_build_") as objdir:
        comp, link = commands(objdir, tmp, quick, extra)
        procs = []
        for cmd in comp:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        failed = False
        for cmd, p in zip(comp, procs):
            log, _ = p.communicate()
            if p.returncode != 0:
                failed = True
                sys.stderr.write(log)
        if failed:
            raise RuntimeError("hipcc failed compiling liblsfft.so")
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking liblsfft.so")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} in {time.time() - t0:.1f}s", flush=True)
    return out


if __name__ == "__main__":
    build(quick="--quick" in sys.argv, verbose=True)
