"""Build libfsz.so (HIP kernels + C ABI) for gfx950, in-tree.

Floating-point flags matter for bit-exactness: -ffp-contract=off keeps every
multiply and add separate; packed fp32 instructions are disabled.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfsz.so")
ARCH = os.environ.get("FSZ_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fsz_kernels.hip", "fsz_api.cpp", "fsz_server.cpp"]

# Kernel-file only: every read-modify-write atomic in the kernels is issued by
# one lane, so the compiler's wave-aggregation rewrite of atomics only adds an
# immediate wait for the result (which also waits for every earlier memory
# operation of the wave, such as in-flight prefetches).
KERNEL_FLAGS = ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        extra = KERNEL_FLAGS if src.endswith(".hip") else []
        cmd = ["hipcc", *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, "hipcc")
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
