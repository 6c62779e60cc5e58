"""Compile the C part of the reference implementation (gcc, OpenMP, -O2, IEEE)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build_c():
    src = os.path.join(HERE, "c", "direct_sum.c")
    out = os.path.join(HERE, "c", "liboracle_direct.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu99",
                           "-o", out, src, "-lm"])
    return out


if __name__ == "__main__":
    print(build_c())
