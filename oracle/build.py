"""Compile the C part of the oracle (test infrastructure) into
oracle/liboracle.so with gcc -O3 -fopenmp."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "direct.c")
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
