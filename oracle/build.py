"""Build the C oracle into a shared library next to its source.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The library is built with
portable flags (no -march=native) because the built file may be copied to a
different host before it is loaded.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "_lb_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile lb_oracle.c with gcc -O3 -fopenmp; return the library path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> str:
    """Return the library path, building it only when no build exists."""
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
