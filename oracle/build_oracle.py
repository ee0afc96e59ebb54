"""Build the BHEM CPU oracle (test infrastructure only) into oracle/liborc.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["patch.cpp", "global.cpp", "capi.cpp", "ray.cpp"]
LIB = os.path.join(HERE, "liborc.so")


def build(extra_flags=(), out=LIB, verbose=False):
    """Compile the oracle with g++ (OpenMP on).  ``extra_flags`` lets a test
    build a variant (e.g. a planted mistake) into another file."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]
    cmd += list(extra_flags)
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True, extra_flags=sys.argv[1:])
