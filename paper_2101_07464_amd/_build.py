"""Build libhd.so (gfx950) in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled
(``-target-feature -packed-fp32-ops``): the kernels accumulate in FP64 and
gain nothing from them.
"""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhd.so")
SOURCES = ["hd_api.hip", "hd_batch.hip", "hd_ista.hip", "hd_kernels.hip",
           "hd_cplx.hip"]
ARCH = "gfx950"


def hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
           "-shared", "-Wall", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC, "-o", tmp]
    cmd += list(extra)
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
