"""Build the HIP library for gfx950 in-tree.

    python -m paper_2609_31258_amd.build

compiles csrc/mc_runtime.hip (single simulations), csrc/mc_server.hip (serving)
and csrc/mc_deposit_op.hip (the stand-alone deposit), which include the
kernels, with hipcc into
paper_2609_31258_amd/libmucite.so.  Flags: -O3, FMA contraction within
each source expression only (-ffp-contract=on: a kernel's rounding then
follows its source, so the single-simulation and the serving kernels, which
inline the same step code, round alike; the kernels turn contraction off
locally where results must be bit-reproducible against plain IEEE
arithmetic), packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmucite.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("mc_runtime.hip", "mc_server.hip", "mc_deposit_op.hip")]
ARCH = os.environ.get("MUCITE_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
           "-I" + os.path.join(ROOT, "include"), "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
