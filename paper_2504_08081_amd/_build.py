"""Build step of libsaltbf.so: hipcc for gfx950, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libsaltbf.so")
SOURCES = ["sb_bandflux.hip", "sb_fit.hip", "sb_probe.hip", "sb_host.cpp", "sb_server.cpp", "sb_nested.cpp"]

# Packed FP32 instructions are switched off for every HIP source.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source and link libsaltbf.so; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + HIP_FLAGS + ["-I", INCLUDE, "-I", CSRC] + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    build_cabi_check(verbose)
    return OUT


CABI_SRC = os.path.join(ROOT, "tests", "c_abi", "sb_cabi_check.cpp")
CABI_EXE = os.path.join(ROOT, "tests", "c_abi", "sb_cabi_check")


def build_cabi_check(verbose: bool = False) -> str:
    """The plain C++ program that drives the C ABI without Python (a test helper), linked
    against the in-tree libsaltbf.so through a relative run path."""
    tmp = CABI_EXE + ".tmp"
    cmd = [hipcc(), "-O2", "-std=c++17", "-Wall", "-I", INCLUDE, CABI_SRC, "-o", tmp, "-L", HERE, "-lsaltbf",
           "-Wl,-rpath,$ORIGIN/../../paper_2504_08081_amd"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, CABI_EXE)
    return CABI_EXE


if __name__ == "__main__":
    print(build(verbose=True))
