"""lc_get_diag_noalloc (diagnostics from a static device scratch array, no
allocation) against lc_get_diag, both called through the C ABI.

Two calls in a row on different contexts, the second on a smaller box (the
static array keeps the first call's partials, which must not leak into the
second), each compared with lc_get_diag on the same state: same kernels and
summation order, so the same bits.  A box larger than the array is refused.
"""
import ctypes
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs

pytestmark = pytest.mark.gpu


def _diag(L, h, fn):
    from paper_1102_2193_amd import lc
    d = lc.Diag()
    rc = getattr(L, fn)(h, 0, ctypes.byref(d))
    assert rc == 0, (fn, rc, L.lc_last_error(h))
    return np.array([d.free_energy, d.mass, d.momentum[0], d.momentum[1], d.momentum[2], d.umax])


def _context(L, precision, steps, seed, a):
    from paper_1102_2193_amd import lc
    ctx = lc.Context([dict(nx=L, precision=precision, **dict(inputs.NEMATIC, q0=2 * math.pi / L))])
    ctx.set_colloid(0, (L / 2 + 0.3, L / 2 - 0.2, L / 2 + 0.1), a, anchoring="planar", W=0.01,
                    vel=(2e-3, 0.0, -1e-3), motion=lc.PRESCRIBED)
    ctx.set_Q(0, inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=seed, noise=0.02))
    ctx.step(steps)
    return ctx


def test_noalloc_diag_matches_diag_on_two_calls():
    from paper_1102_2193_amd import lc
    L = lc.load()
    print("case: no-alloc diagnostics, 48^3 fp32 then 20^3 fp64", flush=True)
    first = _context(48, "fp32", 30, seed=61, a=8.0)
    got1 = _diag(L, first._h, "lc_get_diag_noalloc")
    ref1 = _diag(L, first._h, "lc_get_diag")
    print("   48^3: %s" % got1, flush=True)
    np.testing.assert_array_equal(got1, ref1)
    assert got1[0] != 0.0 and got1[1] > 0.9 * 48 ** 3
    second = _context(20, "fp64", 12, seed=62, a=4.0)
    got2 = _diag(L, second._h, "lc_get_diag_noalloc")
    ref2 = _diag(L, second._h, "lc_get_diag")
    print("   20^3: %s" % got2, flush=True)
    np.testing.assert_array_equal(got2, ref2)
    assert got2[1] < 20 ** 3
    # the first context again, after the smaller call: same bits as before
    np.testing.assert_array_equal(_diag(L, first._h, "lc_get_diag_noalloc"), ref1)
    first.close()
    second.close()


def test_noalloc_diag_refuses_a_box_beyond_the_scratch():
    from paper_1102_2193_amd import lc
    L = lc.load()
    print("case: no-alloc diagnostics refuse a 178^3 box", flush=True)
    ctx = lc.Context([dict(nx=178, precision="fp32", **inputs.NEMATIC)])
    d = lc.Diag()
    rc = L.lc_get_diag_noalloc(ctx._h, 0, ctypes.byref(d))
    assert rc == 1
    assert b"static diagnostics scratch" in L.lc_last_error(ctx._h)
    ctx.close()
