"""Compile the C oracle (test infrastructure) into oracle/liboracle.so with gcc.

Building the checker is not using it: this only runs gcc on msort_oracle.c.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "msort_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def compile_oracle(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-pthread", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(compile_oracle())
