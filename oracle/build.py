"""Build the reference oracle (test infrastructure): one C source, two shared libraries.

liborc_f64.so runs the Kalman part in double, liborc_f32.so in float; the grid and the
neighbour links are binary32 in both.  -ffp-contract=off keeps every product and sum
separately rounded, as the binary32 steps require.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def lib_path(mode: str) -> str:
    return os.path.join(HERE, f"liborc_{mode}.so")


def build(verbose: bool = False) -> None:
    for mode, defs in (("f64", []), ("f32", ["-DORC_FP32"])):
        out = lib_path(mode)
        cmd = ["gcc", *FLAGS, *defs, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
