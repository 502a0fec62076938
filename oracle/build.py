"""Build the FP64 CPU oracle (``liblco.so``) with gcc.

Test infrastructure only: the oracle is the checker of the HIP library and
is built next to it, never linked into it.

With LCO_SANITIZE=1 in the environment the oracle is built as
``liblco_san.so`` with the address and undefined-behaviour sanitizers (any
report aborts); the process must then preload the sanitizer runtime, e.g.

    LCO_SANITIZE=1 LD_PRELOAD=$(gcc -print-file-name=libasan.so) \
    ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu" -k oracle
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lco.c")
SANITIZE = os.environ.get("LCO_SANITIZE", "") not in ("", "0")
LIB = os.path.join(HERE, "liblco_san.so" if SANITIZE else "liblco.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(force: bool = True) -> str:
    """Compile oracle/lco.c into the oracle library; returns its path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    opt = SAN_FLAGS if SANITIZE else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
                           SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
