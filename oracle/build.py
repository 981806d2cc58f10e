"""Build the CPU oracle (test infrastructure) with gcc.

    python oracle/build.py

Plain C99, -O2 -ffp-contract=off (no contraction: every multiply-add is
rounded as written, and the one fused multiply-add in the sampling
specification is an explicit fma call), OpenMP for the loop over independent
amplitude groups.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "sv_oracle.c")
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
