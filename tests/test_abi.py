"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/lc.h, and rejects invalid parameters before touching the
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "lc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1102_2193_amd import lc
    if not os.path.exists(lc.LIB_PATH):
        pytest.fail("liblc.so is not built; run __graft_entry__.build()")
    return lc.load()


def test_header_declares_the_core_calls():
    names = declared()
    for n in ("lc_create", "lc_set_colloid", "lc_step", "lc_get_Q", "lc_get_force"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1102_2193_amd import lc
    names = declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lc.EXPORTS) == names


def test_struct_sizes_match_header(lib, tmp_path):
    # the ctypes structures against the C header itself (sizes and offsets
    # printed by a program compiled from include/lc.h)
    import subprocess
    from paper_1102_2193_amd import lc
    from paper_1102_2193_amd import nn
    structs = {"lc_params": lc.Params, "lc_colloid": lc.Colloid, "lc_diag": lc.Diag, "lc_nn_case": nn.Case}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lc.h"', '#include "lc_nn.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.parametrize("field,value", [("nx", 4), ("tau", 0.5), ("precision", 7), ("rho0", 0.0),
                                         ("Gamma", -1.0)])
def test_create_rejects_bad_parameters(lib, field, value):
    from paper_1102_2193_amd import lc
    p = lc.make_params(16)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    rc = lib.lc_create(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == 1 and not h.value
    assert lib.lc_last_error(None)


def test_batch_rejects_mixed_precision(lib):
    from paper_1102_2193_amd import lc
    arr = (lc.Params * 2)(lc.make_params(16, precision=lc.FP32), lc.make_params(16, precision=lc.FP64))
    h = ctypes.c_void_p()
    assert lib.lc_create_batch(2, arr, None, ctypes.byref(h)) == 1
    assert b"precision" in lib.lc_last_error(None)


def test_null_context_calls_fail_cleanly(lib):
    assert lib.lc_step(None, 1) == 1
    assert lib.lc_sync(None) == 1
    assert lib.lc_get_nstep(None) == -1


def test_nn_header_symbols_exported(lib):
    from paper_1102_2193_amd import nn
    src = open(os.path.join(ROOT, "include", "lc_nn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(lc_nn_[A-Za-z0-9_]+)\s*\(", src)))
    assert names == sorted(nn.EXPORTS)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert ctypes.sizeof(nn.Case) == 8 * 3 + 8 + 8 + 4 + 4 + 8 + 8


def test_nn_create_rejects_bad_grid(lib):
    from paper_1102_2193_amd import nn
    L = nn._lib()
    h = ctypes.c_void_p()
    assert L.lc_nn_create(12, 0, None, ctypes.byref(h)) == 1
    assert b"multiple of 8" in L.lc_nn_last_error(None)
    # the elementwise kernels index voxels in 32 bits
    assert L.lc_nn_create(1032, 0, None, ctypes.byref(h)) == 1
    assert b"[8, 1024]" in L.lc_nn_last_error(None)
