"""Compiles the CPU oracle (oracle.cpp) into oracle/liboracle.so, and the same source a second
time into oracle/liboracle_fast.so for the timed CPU baseline.

Test infrastructure: the oracle is built so that tests, the smoke check and the benchmark's
CPU baseline can run it; the product library never links or loads it.
liboracle.so (every parity reference): floating-point contraction off, so that the
differential-evolution arithmetic rounds each operation separately.  liboracle_fast.so (only its
double-precision synthesis and evolution are called, to time the baseline): -O3 for AVX2/FMA
x86-64 (x86-64-v3) with contraction allowed.  No fast-math flag is used anywhere.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_FAST = os.path.join(HERE, "liboracle_fast.so")

FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas"]
FAST_FLAGS = ["-O3", "-march=x86-64-v3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=fast",
              "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas"]


def _compile(flags, out):
    tmp = out + ".tmp"
    subprocess.run(["g++", *flags, SRC, "-o", tmp, "-lquadmath"], check=True)
    os.replace(tmp, out)


SANITIZE_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                  "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                  "-Wno-unknown-pragmas"]


def build_sanitized(out: str) -> str:
    """The parity build's arithmetic with AddressSanitizer and UndefinedBehaviorSanitizer, into
    `out` (host code only; loaded by a process that preloads the sanitizer runtimes)."""
    _compile(SANITIZE_FLAGS, out)
    return out


def build(force: bool = True) -> str:
    for flags, out in ((FLAGS, LIB), (FAST_FLAGS, LIB_FAST)):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            _compile(flags, out)
    return LIB


if __name__ == "__main__":
    print(build())
