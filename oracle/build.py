"""Build the CPU oracle's shared library (test infrastructure only).

Compiles ``cse_oracle.c`` with the host C compiler into ``libcse_oracle.so``
next to this file.  Run by the repository's build entry point; importing the
oracle wrapper never compiles anything.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cse_oracle.c")
LIB = os.path.join(HERE, "libcse_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", LIB + ".tmp", SRC, "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
