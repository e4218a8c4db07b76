"""Build the plain-C oracle into oracle/liboracle.so with gcc.

Test infrastructure: the oracle is the independent checker of the GPU
library and is never linked into it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")


def build(out=LIB_PATH, src=SRC, extra=()):
    """Compile `src` to the shared library `out` (always recompiles)."""
    tmp = out + ".tmp"
    # float arithmetic exactly as written: one rounding per operation
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-fPIC", "-shared",
           *extra, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
