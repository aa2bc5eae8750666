"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled with gcc, contraction of a*b+c into fma
disabled, no fast-math, round-to-nearest-even (switched to rounding toward
-infinity only around the one product that asks for it, hence
-frounding-math), gradual underflow.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["ora_evd2.c", "ora_sevd2.c", "ora_svd.c", "ora_ssvd.c", "ora_nrmf.c", "ora_exact.c"]
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only", "-frounding-math",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-D_GNU_SOURCE"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-o", tmp] + [os.path.join(HERE, s) for s in SOURCES] + ["-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
