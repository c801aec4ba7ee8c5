"""Compile the C oracle (FP64 sweep, adjoint, light-cone boxes) and the C
bit-level arithmetic model into one shared library next to this file (gcc,
OpenMP, no contraction of multiplies and adds).  Test infrastructure: see
``oracle/__init__.py``."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "so2dr_oracle.c"), os.path.join(HERE, "emulator_bits.c")]
OUT = os.path.join(HERE, "libso2dr_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off"] + SRCS + ["-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
