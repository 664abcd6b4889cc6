"""Builds liboracle.so (plain C, gcc).  TEST INFRASTRUCTURE ONLY.

Compiled with -ffp-contract=off so that every binary64 operation rounds
exactly where the C source says; fma() is called explicitly where the codec
definition uses a fused multiply-add.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["codec.c", "mpm.c", "adjoint.c"]
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", OUT + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
