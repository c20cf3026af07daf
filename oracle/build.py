"""Compile the CPU oracle (test infrastructure only) into oracle/_fcfc_oracle.so.

Flags: -O2 without -march (no FMA instructions), -ffp-contract=off so that no
multiply-add is ever fused, -fno-fast-math, OpenMP for the outer loop.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fcfc_oracle.c")
LIB = os.path.join(HERE, "_fcfc_oracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(force=True, src=SRC, out=LIB, extra=()):
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
