"""Build the CPU oracle library (test infrastructure only).

``python oracle/build.py`` compiles ``tor_oracle.c`` with gcc into
``oracle/libtororacle.so``.  Plain IEEE arithmetic: no fast-math, no FMA
contraction, so every operation rounds as the C source reads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tor_oracle.c")
LIB = os.path.join(HERE, "libtororacle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-variable", "-pthread",
           SRC, "-o", LIB + ".tmp", "-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
