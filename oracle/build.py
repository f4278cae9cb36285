"""Build the oracle shared library with gcc (plain C, -O2, no fast-math).

TEST INFRASTRUCTURE ONLY: the oracle is loaded by the test suite, the smoke
check and the benchmark's CPU-baseline leg, never by the library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["domain.c", "mlp.c", "search.c", "search_real.c", "train.c"]
OUT = os.path.join(HERE, "_build", "liboracle.so")


def build(verbose=False):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-fno-fast-math", "-ffp-contract=off", "-pthread", "-o", OUT + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
