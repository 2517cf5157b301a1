"""Build the oracle library (plain C, FP64) with gcc.

Test infrastructure: the oracle is only loaded by the tests, the smoke check
and the CPU-baseline leg of the benchmark.  Contraction is off and no
fast-math flag is used so that every floating-point operation is the one
written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mbt_ref.c")
LIB = os.path.join(HERE, "libmbt_ref.so")

CFLAGS = ["-std=c11", "-O2", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built():
    """Build once if the library is missing or older than its source."""
    if (not os.path.exists(LIB)) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "mbt_ref.h"))):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
