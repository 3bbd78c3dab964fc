"""Compile the oracle's C source into oracle/liblst_oracle.so (plain gcc, FP64,
no FMA contraction so results follow the written operation order)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblst_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lst_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wno-unused-function", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
