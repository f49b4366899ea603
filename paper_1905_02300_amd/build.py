"""Build libyy.so (gfx950) in-tree with hipcc.

Compiles every HIP/C++ source under csrc/ with -O3 for gfx950 only,
without packed-FP32 instructions, and links one shared library next to
this file.  Multiply-adds are fused only within one source expression
(-ffp-contract=on), so that a kernel body rounds alike in every kernel it
is instantiated in (the one-shell kernels and the batched ones).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libyy.so")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# (source, extra flags, object): the kernels are compiled once per compute
# precision, so that the two halves build in parallel
UNITS = [("yy_kernels.hip", ["-DYY_ONLY_DOUBLE"], "yy_kernels_f64.o"),
         ("yy_kernels.hip", ["-DYY_ONLY_FLOAT"], "yy_kernels_f32.o"),
         ("yy_host.cpp", [], "yy_host.o"),
         ("yy_static.hip", [], "yy_static.o")]


def build(verbose=False):
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    procs, objs = [], []
    for src, extra, obj in UNITS:
        obj = os.path.join(HERE, "_build", obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc", *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
