"""Build the CPU oracle libraries (test infrastructure; g++ only, no HIP).

liboracle.so holds the explicit hydro step (hydro_oracle.cpp) and
libfld_oracle.so the implicit radiation diffusion step with its multigrid
solver (fld_oracle.cpp).  Both are compiled with -ffp-contract=off so that
every multiply and add rounds separately, in the order the source states.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "hydro_oracle.cpp")]
FLD_LIB = os.path.join(HERE, "libfld_oracle.so")
FLD_SRC = [os.path.join(HERE, "fld_oracle.cpp")]


SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]
ASAN_LIB = os.path.join(HERE, "liboracle_asan.so")
ASAN_FLD_LIB = os.path.join(HERE, "libfld_oracle_asan.so")


def _compile(srcs, out, verbose, extra=()):
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", *extra, "-o", out + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False, src=None, out=None) -> str:
    """Compile hydro_oracle.cpp (or `src`) into liboracle.so (or `out`); with
    no `src`, also compile fld_oracle.cpp into libfld_oracle.so."""
    if src is None:
        _compile(FLD_SRC, FLD_LIB, verbose)
    return _compile([src] if src else SRC, out or LIB, verbose)


def build_sanitized(verbose: bool = False):
    """AddressSanitizer + UndefinedBehaviorSanitizer builds of both oracle
    libraries (liboracle_asan.so, libfld_oracle_asan.so).  A process that
    loads them needs gcc's libasan (first) and libubsan in LD_PRELOAD; the
    oracle modules load them instead of the plain builds when the environment
    names them in HARD_ORACLE_LIB and HARD_FLD_ORACLE_LIB."""
    _compile(SRC, ASAN_LIB, verbose, SAN_FLAGS)
    _compile(FLD_SRC, ASAN_FLD_LIB, verbose, SAN_FLAGS)
    return ASAN_LIB, ASAN_FLD_LIB


def build_fld(verbose: bool = False, src=None, out=None) -> str:
    """Compile fld_oracle.cpp (or `src`) into libfld_oracle.so (or `out`)."""
    return _compile([src] if src else FLD_SRC, out or FLD_LIB, verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
