"""Build the CPU oracle shared library (test infrastructure; gcc, OpenMP).

Only the tests, the smoke check and the benchmark's CPU-baseline leg load the result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["or_params.c", "or_lattice.c", "or_zuker.c", "or_eval.c", "or_brute.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(extra_flags=()):
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-Wno-unused-parameter", *extra_flags,
           *[os.path.join(HERE, s) for s in SOURCES], "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(sys.argv[1:]))
