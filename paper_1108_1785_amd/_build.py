"""Compile libgnm.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgnm.so")
SOURCES = ["registry.cpp", "kernels.hip", "hist.hip", "hosts.hip", "table.hip", "forms.cpp", "ingest.hip"]
HEADERS = [os.path.join(INCLUDE, "gnm.h"), os.path.join(CSRC, "gnm_internal.h"),
           os.path.join(CSRC, "registry.h"), os.path.join(CSRC, "gnm_device.h"), os.path.join(CSRC, "hist.h"),
           os.path.join(CSRC, "hosts.h"),
           os.path.join(CSRC, "partition.h"), os.path.join(CSRC, "table.h")]

# Packed FP32 instructions are kept off for every device pass.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Always recompiles (the build check must exercise the compiler)."""
    objs = []
    cc = hipcc()
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, s + ".o")
        cmd = [cc] + COMMON + DEVICE_FLAGS + ["-c", src, "-o", obj]
        if s.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
