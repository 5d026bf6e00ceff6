"""Build the C oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, no contraction of floating-point expressions, OpenMP over
independent source nodes.  Called by __graft_entry__.build() and, lazily, by
the oracle loader when the library is missing.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cl_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=gnu99", "-Wall", "-Wextra",
        "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
