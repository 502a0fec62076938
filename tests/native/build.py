"""Build the C driver of the library's ABI (tests/native/lc_abi_run.c).

``build()`` links it against paper_1102_2193_amd/liblc.so (run by
tests/test_native_gpu.py); ``build(host_sanitize=True)`` links it against
liblc_hostsan.so with clang's address and undefined-behaviour sanitizers,
so the library's host code runs under them with nothing preloaded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1102_2193_amd")
SRC = os.path.join(HERE, "lc_abi_run.c")
EXE = os.path.join(HERE, "lc_abi_run")
EXE_HOSTSAN = os.path.join(HERE, "lc_abi_run_hostsan")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(host_sanitize: bool = False) -> str:
    exe = EXE_HOSTSAN if host_sanitize else EXE
    lib = "liblc_hostsan.so" if host_sanitize else "liblc.so"
    cc = [CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] if host_sanitize \
        else ["gcc", "-O2"]
    cmd = cc + ["-std=c11", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"), SRC, "-L", PKG, "-l:" + lib,
                "-Wl,-rpath,$ORIGIN/../../paper_1102_2193_amd", "-lm", "-o", exe]
    subprocess.run(cmd, check=True)
    return exe


if __name__ == "__main__":
    print(build(host_sanitize="--host-sanitize" in sys.argv[1:]))
