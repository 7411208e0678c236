"""Build libdfa.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1506_08612_amd.build [--isa DIR]
"""
from __future__ import annotations

import argparse
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdfa.so")
ARCH = "gfx950"

# Packed-FP32 instructions are kept out of every code object (no float math on
# this path, but the flag holds for all HIP code built here).
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def host_cxx() -> str:
    for c in (os.environ.get("CXX"), shutil.which("g++"), "/opt/rocm/llvm/bin/clang++"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("no host C++ compiler found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, isa_dir: str | None = None) -> str:
    """Compile every source under csrc/ into paper_1506_08612_amd/libdfa.so."""
    cc = hipcc()
    objs = []
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [cc, *HIP_FLAGS, "-c", src, "-o", obj]
        if src.endswith(".cpp"):
            # host-only sources: the host compiler, no device code object
            cmd = [host_cxx(), "-O2", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC,
                   "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
        if isa_dir and src.endswith(".hip"):
            os.makedirs(isa_dir, exist_ok=True)
            out = os.path.join(isa_dir, os.path.basename(src) + ".s")
            subprocess.check_call([cc, *HIP_FLAGS, "--cuda-device-only", "-S", src, "-o", out])
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--isa", default=None, help="also write device assembly here")
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args(argv)
    print(build(verbose=a.v, isa_dir=a.isa))


if __name__ == "__main__":
    sys.exit(main())
