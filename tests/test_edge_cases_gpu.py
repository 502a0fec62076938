"""Degenerate and limiting cases of the step, against the oracle.

* The smallest boxes the library takes (edges of 8 sites), narrower than
  every tile shape: 8^3 with the largest colloid that fits one (a = 2, the
  box edge being at least 2a + 4), planar anchoring, chiral, moving across
  the periodic corner so that nodes change side (the moving-boundary events
  of Sec. 2.2), at the paper's parameters with tau = 0.8; and a ragged
  8 x 9 x 11 box without colloid.  Every tile shape of both precisions.
* Zero steps: the state is left as it was set and the step count stays 0.
* The smallest colloid (a just above 1, centred between nodes): eight solid
  nodes, every one a boundary node with fluid neighbours, none interior.

Bounds as in the other parity tests: FP64 to round-off, FP32 to 1e-5 on Q
and f and 1e-3 on the force history.
"""
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs
from test_parity_gpu import check, run_pair, say

pytestmark = pytest.mark.gpu

PAPER = dict(inputs.PAPER_CHOLESTERIC)


def _tiles(precision):
    from paper_1102_2193_amd import lc
    ctx = lc.Context([dict(nx=8, precision=precision, **inputs.NEMATIC)])
    shapes = [tuple(ctx.tile_shape(t)) for t in range(ctx.num_tiles())]
    ctx.close()
    return shapes


def _check(r, precision, colloid):
    if precision == "fp64":
        check(r, 1e-10, 1e-12, tol_u=1e-8, tol_force=1e-8 if colloid else None)
    else:
        check(r, 1e-5, 1e-5, tol_force=1e-3 if colloid else None)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_smallest_box_every_tile(precision):
    L, n = 8, 30
    prm = dict(PAPER, tau=0.8, q0=2 * math.pi / 8)
    col = dict(pos=(7.4, 0.3, 7.8), a0=2.0, anchoring="planar", W=0.05, S0=0.5, motion=1,
               vel=(0.03, -0.02, 0.025), omega=(0.0, 0.01, 0.0))
    Q0 = inputs.noisy_nematic_q(L, L, L, 0.5, seed=61, noise=0.02, director=(1, 0.2, 0.4))
    Qr = inputs.noisy_nematic_q(8, 9, 11, 0.5, seed=62, noise=0.02, director=(0.3, 1, 0.2))
    for tile, shape in enumerate(_tiles(precision)):
        say("case: 8^3 %s tile %s, a = 2 moving across the corner, %d steps" % (precision, shape, n))
        r = run_pair((L, L, L), prm, n, precision, colloid=col, Q0=Q0, tile=tile, hist=True)
        _check(r, precision, True)
        assert r["ctx"].solid_id(0).sum() > 0
        np.testing.assert_array_equal(np.array(r["ctx"].get_colloid(0).pos), np.array(r["ref"].get_colloid().pos))
        r["ctx"].close()
        say("case: 8x9x11 %s tile %s, no colloid, %d steps" % (precision, shape, n))
        r = run_pair((8, 9, 11), prm, n, precision, Q0=Qr, tile=tile)
        _check(r, precision, False)
        r["ctx"].close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_steps_leave_the_state(precision):
    from paper_1102_2193_amd import lc
    say("case: 16^3 %s, step(0)" % precision)
    L = 16
    ctx = lc.Context([dict(nx=L, precision=precision, **inputs.NEMATIC)])
    ctx.set_colloid(0, (8.2, 7.9, 8.4), 3.0, anchoring="normal", W=math.inf, S0=0.5)
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=63, noise=0.01)
    ctx.set_Q(0, Q0)
    Q1, f1, u1 = ctx.get_Q(0), ctx.get_f(0), ctx.get_u(0)
    ctx.step(0)
    assert ctx.nstep == 0
    np.testing.assert_array_equal(ctx.get_Q(0), Q1)
    np.testing.assert_array_equal(ctx.get_f(0), f1)
    np.testing.assert_array_equal(ctx.get_u(0), u1)
    fluid = ctx.solid_id(0) == 0
    dt = np.float32 if precision == "fp32" else np.float64
    np.testing.assert_array_equal(Q1[:, fluid], Q0.astype(dt).astype(np.float64)[:, fluid])
    with pytest.raises(lc.LCError):
        ctx.step(-1)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_smallest_colloid_has_no_interior(precision):
    L, n = 16, 40
    col = dict(pos=(7.5, 8.5, 7.5), a0=1.01, anchoring="normal", W=0.02, S0=0.5)
    say("case: 16^3 %s, a = 1.01 between nodes (8 solid nodes), %d steps" % (precision, n))
    Q0 = inputs.noisy_nematic_q(L, L, L, 0.5, seed=64, noise=0.02, director=(1, 0.2, 0.4))
    r = run_pair((L, L, L), dict(PAPER, tau=0.8), n, precision, colloid=col, Q0=Q0, hist=True)
    solid = r["ctx"].solid_id(0) > 0
    assert solid.sum() == 8 and np.array_equal(solid, ~r["fluid"])
    _check(r, precision, True)
    assert np.linalg.norm(r["Hr"][-1]) > 0
    r["ctx"].close()
