"""Build the FP64 CPU oracle (plain C, gcc, libm) into oracle/liboracle.so.

Test infrastructure: the oracle is compiled with -ffp-contract=off and no
fast-math so that its arithmetic is the plain IEEE sequence written in the
source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "mcv_oracle.c")
    tmp = f"{LIB}.{os.getpid()}.tmp"  # concurrent builds never share a file
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
