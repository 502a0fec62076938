"""Build the HIP library ``liblc.so`` for gfx950 with hipcc (in-tree).

``python build.py --host-sanitize`` builds ``liblc_hostsan.so`` instead: the
host code (runtime, launchers, bindings) with the address and
undefined-behaviour sanitizers, the device code unchanged.  Load it with
LC_LIBRARY pointing at it and clang's ASan runtime preloaded, e.g.

    LC_LIBRARY=$PWD/paper_1102_2193_amd/liblc_hostsan.so ASAN_OPTIONS=detect_leaks=0 \
    LD_PRELOAD=/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so python -m pytest tests -m gpu
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblc.so")
LIB_HOSTSAN = os.path.join(HERE, "liblc_hostsan.so")
SOURCES = ["lc_kernels.hip", "lc_runtime.hip", "nn_kernels.hip", "nn_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         # packed FP32 instructions are disabled on purpose
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]
# sanitizers on the host pass only (each flag right after -Xarch_host)
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer -Xarch_host -g").split()


def build(verbose: bool = False, host_sanitize: bool = False) -> str:
    """Compile every source and link liblc.so (liblc_hostsan.so with
    host_sanitize); returns the library path."""
    objs = []
    procs = []
    extra = HOST_SAN if host_sanitize else []
    lib = LIB_HOSTSAN if host_sanitize else LIB
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".hostsan.o" if host_sanitize else ".o"))
        cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    for p, src in procs:
        _, err = p.communicate()
        err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, err))
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + extra + objs + ["-o", tmp], check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, host_sanitize="--host-sanitize" in sys.argv[1:]))
