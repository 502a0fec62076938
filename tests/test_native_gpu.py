"""The library driven from plain C through include/lc.h alone.

tests/native/lc_abi_run.c (built by __graft_entry__.build()) creates FP32
and FP64 contexts, one and several colloids with the variants, a batch on
every tile shape, steps with and without graphs, reads every field and
diagnostic, checkpoints and restarts bit for bit, and checks the documented
error returns.  It must exit 0.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "lc_abi_run")


def test_c_driver_of_the_abi():
    assert os.path.exists(EXE), "tests/native/lc_abi_run is not built; run __graft_entry__.build()"
    print("case: C driver of the ABI", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=240)
    print(r.stdout)
    assert r.returncode == 0, "C driver failed (rc %d):\n%s\n%s" % (r.returncode, r.stdout[-3000:], r.stderr[-6000:])
