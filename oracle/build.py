"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle_hd.so.

Plain C11 at -O3 with IEEE semantics (no fast-math, which would let the
compiler reorder the floating-point sums; no -march, so the library built here
runs on any x86-64 host).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "hd_oracle.c"),
        os.path.join(HERE, "hd_cplx_oracle.c")]
LIB = os.path.join(HERE, "liboracle_hd.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
