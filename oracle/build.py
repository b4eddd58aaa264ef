"""Build the oracle's C sparse LU (plain gcc, no GPU code).

TEST INFRASTRUCTURE ONLY: the oracle is compiled here so that the checker
exists wherever the tests run; the solver library never links it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "_splu.so")


def build(force: bool = True) -> str:
    src = os.path.join(HERE, "splu.c")
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(src):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
