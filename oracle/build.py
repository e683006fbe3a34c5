"""Build the oracle's C part (O1, the direct DFT) with gcc.

TEST INFRASTRUCTURE ONLY: compiles oracle/dft.c into
oracle/_build/libwgoracle.so.  FP contraction is switched off so that every
FP64 operation is individually rounded.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libwgoracle.so")


def build(force=True):
    os.makedirs(OUT_DIR, exist_ok=True)
    src = os.path.join(HERE, "dft.c")
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(src):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-std=c11", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
