"""Compiles the CPU oracle (oracle.cpp) into oracle/liboracle.so.

Test infrastructure: the oracle is built so that tests, the smoke check and the benchmark's
CPU baseline can run it; the product library never links or loads it.
Floating-point contraction is off so that the differential-evolution arithmetic rounds each
operation separately, and no fast-math flag is used anywhere.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["g++", *FLAGS, SRC, "-o", tmp, "-lquadmath"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
