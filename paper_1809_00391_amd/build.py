"""Build libmbt.so (the HIP tracker behind include/mbt.h) for gfx950 in-tree.

hipcc cross-compiles without a GPU.  Device code is built with floating-point
contraction off (every multiply and add is the one written, so coordinate
arithmetic matches a plain FP64 reference operation for operation) and with
packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmbt.so")
SOURCES = [os.path.join(CSRC, "mbt_kernels.hip"), os.path.join(CSRC, "mbt_host.cpp")]
HEADERS = [os.path.join(CSRC, "mbt_internal.h"), os.path.join(CSRC, "mbt_fastmath.h"),
           os.path.join(CSRC, "mbt_rw.h"),
           os.path.join(INCLUDE, "mbt.h")]
ARCH = os.environ.get("MBT_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def build(verbose=False):
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC, *lang, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
