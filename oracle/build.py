"""Compile the plain-C FP64 oracle (test infrastructure) into liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ("sfpic_oracle.c", "sfpic_oracle3d.c")


def build(force: bool = True) -> str:
    srcs = [os.path.join(HERE, f) for f in SOURCES]
    if force or not os.path.exists(LIB) or any(
            os.path.getmtime(LIB) < os.path.getmtime(s) for s in srcs):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
                               "-fPIC", "-shared", "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
