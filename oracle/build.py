"""Build the float64 CPU oracle library (test infrastructure only).

Compiles ``gpair_oracle.c`` with gcc into ``libgpair_oracle.so`` next to this
file.  Portable x86-64 code (no -march=native: the library is built in one
container and run on other hosts), OpenMP for the sensor/kernel loops and
``-ffp-contract=off`` so every float64 operation is rounded separately.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gpair_oracle.c")
LIB = os.path.join(HERE, "libgpair_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
