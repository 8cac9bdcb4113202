"""Build the CPU oracle shared library (test infrastructure only).

Plain C99, ``-O2`` without fast-math, so every operation rounds as IEEE
double precision says.  Invoked by ``__graft_entry__.build()``; tests load
the result through ``oracle/__init__.py``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["philox.c", "physics.c", "transport.c", "field.c", "csg.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fno-fast-math",
           "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
