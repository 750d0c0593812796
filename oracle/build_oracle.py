"""Compile the C part of the oracle (test infrastructure) into oracle/liboracle_sw.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sw_oracle.c")
LIB = os.path.join(HERE, "liboracle_sw.so")
CFLAGS = ["-O2", "-std=c99", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
