"""Build the CPU oracle library (oracle/liboracle.so) with gcc.

Test infrastructure: the oracle is the plain FP64 CPU reference that the GPU
path is checked against; building it is part of building the checker.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
