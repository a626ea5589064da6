"""Compile the oracle's C helper (oracle/csrc/pairs.c -> oracle/_pairs.so)
with gcc.  Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "pairs.c")
OUT = os.path.join(HERE, "_pairs.so")


def build(verbose=False):
    cmd = ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
