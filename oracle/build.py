"""Build the FP64 CPU oracle (test infrastructure) as a shared library with gcc.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
the result.  Plain IEEE arithmetic: no -ffast-math, no host-specific -march,
so the library built here also runs on another x86-64 host.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hbref.c")
LIB = os.path.join(HERE, "libhbref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
