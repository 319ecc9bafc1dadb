"""Build libtpcsf.so (HIP, gfx950) in-tree.

Flags: -O3; packed-FP32 instructions disabled (the hand-written binary32 stages rely on
ordinary scalar rounding, and the compiler's packed forms are avoided altogether); the
binary32 grid and link stages turn contraction off in their own scope, so no global
-ffp-contract flag is needed.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", f) for f in ("tpcsf_kernels.hip", "tpcsf_merge.hip", "tpcsf_compress.hip", "tpcsf_host.hip",
                                                        "tpcsf_server.hip")]
LIB = os.path.join(PKG, "libtpcsf.so")
ARCH = os.environ.get("TPCSF_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmd = [hipcc, *FLAGS, *extra, "-o", LIB + ".tmp", *SRC]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
