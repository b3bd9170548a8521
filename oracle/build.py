"""Build step for the CPU oracle (test infrastructure only).

Compiles ``szref.c`` into ``libszref.so`` next to it with the host compiler:
C11, -O2, no FMA contraction, no fast-math, SSE floating point (no x87 excess
precision), so that every step rounds once in the element type.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libszref.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
        "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse",
        "-fPIC", "-shared", "-o", LIB + ".tmp", os.path.join(HERE, "szref.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
