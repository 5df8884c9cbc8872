"""Builds the FP64 CPU oracle library (test infrastructure only).

Compiled with gcc, contraction of a*b+c into fused multiply-adds disabled so
every expression is evaluated in the order written, and no host-specific
instruction set so the library runs on any x86-64 host.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    src = os.path.join(HERE, "schw_oracle.c")
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(src):
        return LIB
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-o", LIB + ".tmp", src, "-lm"]
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
