"""Build the CPU oracle library (test infrastructure; g++ only, no HIP).

The oracle is compiled with -ffp-contract=off so that every multiply and add
rounds separately, in the order the source states.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "hydro_oracle.cpp")]


def build(verbose: bool = False, src=None, out=None) -> str:
    """Compile hydro_oracle.cpp (or `src`) into liboracle.so (or `out`)."""
    out = out or LIB
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", out + ".tmp"] + ([src] if src else SRC)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
