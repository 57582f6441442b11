"""Build the CPU oracle shared library (test infrastructure).

    python -m oracle.build

compiles mc_oracle.c with gcc -O2 -ffp-contract=off -fopenmp into
oracle/libmc_oracle.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmc_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "mc_oracle.c")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
           "-shared", "-fPIC", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
