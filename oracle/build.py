"""Build the C oracle (test infrastructure) into shared libraries next to this file.

    libtlbref64.so  -- the FP64 oracle
    libtlbref32.so  -- the same source with every operation in FP32 (error envelope only)

gcc, -O2, OpenMP over theta rows, and -ffp-contract=off so that the compiler fuses no
multiply-add: the oracle's rounding follows its source text.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tlb_oracle.c")


def lib_path(bits=64):
    return os.path.join(HERE, f"libtlbref{bits}.so")


def build(verbose=False):
    for bits, real in ((64, "double"), (32, "float")):
        out = lib_path(bits)
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
               f"-DTLBREF_REAL={real}", SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
