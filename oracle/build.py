"""Builds the FP64 CPU oracle (test infrastructure only) with gcc.

    python oracle/build.py            # -> oracle/liblbm_oracle.so

The oracle is plain C compiled with -O2; OpenMP parallelises the per-node
loops (the results do not depend on the thread count: every parallel loop
writes disjoint elements and all sums run serially).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lbm_oracle.c", "conv_oracle.c"]
OUT = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wno-unused-function", "-o", OUT + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
