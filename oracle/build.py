"""Compile the FP64 oracle (test infrastructure) into oracle/libtcol_oracle.so with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tcol_oracle.c")
LIB = os.path.join(HERE, "libtcol_oracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off: no fused multiply-adds, so every product is rounded as written
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
