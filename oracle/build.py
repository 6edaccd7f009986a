"""Build the CPU oracle library (plain C, gcc, OpenMP).

Test infrastructure: only the test suite, the smoke check and the benchmark's
CPU-baseline leg load what this builds.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libffsoracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "ffs_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
