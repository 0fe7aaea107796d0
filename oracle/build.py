"""Builds the FP64 CPU oracle (test infrastructure only) with gcc.

    python oracle/build.py            # -> oracle/liblbm_oracle.so

The oracle is plain C compiled with -O2; OpenMP parallelises the per-node
loops (the results do not depend on the thread count: every parallel loop
writes disjoint elements and all sums run serially).  ``native=True`` builds
a copy with -O3 -march=native for the machine it runs on (the CPU timing
baseline and long golden runs); ISO C mode keeps floating-point contraction
off, so both builds give the same bits.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lbm_oracle.c", "conv_oracle.c"]
OUT = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False, out: str = OUT, native: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
                           "-Wall", "-Wno-unused-function", "-o", out + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
