"""Build libfv.so in-tree with hipcc for gfx950.

The library is every HIP kernel source plus the C++ host runtime in csrc/,
linked into one shared object next to this file.  `python -m
paper_2501_13051_amd.build` rebuilds it.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfv.so")
ARCH = os.environ.get("FV_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))), sorted(glob.glob(os.path.join(CSRC, "*.cpp")))


def _run(cmd, verbose):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libfv.so")
    if verbose:
        sys.stderr.write(res.stderr)


def build(verbose: bool = False) -> str:
    """Compile each source to an object (device code for gfx950 only), then
    link the shared library."""
    hip_srcs, cpp_srcs = sources()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = "-I" + os.path.join(ROOT, "include")
    objs = []
    for src in hip_srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        _run([hipcc(), "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              # packed fp32 ops stay off in all device code
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              inc, "-c", src, "-o", obj], verbose)
        objs.append(obj)
    for src in cpp_srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        _run([hipcc(), "-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", inc,
              "-c", src, "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
