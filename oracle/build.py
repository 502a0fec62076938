"""Build the FP64 CPU oracle (``liblco.so``) with gcc.

Test infrastructure only: the oracle is the checker of the HIP library and
is built next to it, never linked into it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lco.c")
LIB = os.path.join(HERE, "liblco.so")


def build(force: bool = True) -> str:
    """Compile oracle/lco.c into oracle/liblco.so; returns the library path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
           SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
