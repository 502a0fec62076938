"""Several colloids per box on the GPU against the oracle (the colloid-colloid
interactions of the paper's outlook, Introduction and Sec. 3.2).

Fixed, prescribed (with moving-boundary events) and free colloids, two and
three per box, nematic and chiral, with and without the higher-order
variants.  FP64 to round-off on the fields and on every colloid's force
history; FP32 to 1e-5 on Q and f and 1e-3 on the forces.  Also: the
library's solid map, the separation rule, checkpoints and a batch whose
boxes hold different numbers of colloids.
"""
import ctypes
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs
from test_parity_gpu import ANCH, rel_inf, rel_l2, say

pytestmark = pytest.mark.gpu

NEM = inputs.NEMATIC


def _oracle_specs(specs):
    out = []
    for sp in specs:
        o = dict(sp)
        o["anchoring"] = ANCH[o.get("anchoring", "normal")]
        out.append(o)
    return out


def run_multi(L, prm, steps, precision, specs, Q0, tile=None):
    from oracle import lco
    from paper_1102_2193_amd import lc
    ctx = lc.Context([dict(nx=L, precision=precision, **prm)])
    ctx.set_colloids(0, specs)
    if tile is not None:
        ctx.set_tile(tile)
    ctx.set_Q(0, Q0)
    ctx.step(steps)
    ref = lco.Sim(L, **prm)
    ref.set_colloids(_oracle_specs(specs))
    ref.set_Q(Q0)
    hist = []
    for _ in range(steps):
        ref.step(1)
        hist.append(ref.forces())
    n = len(specs)
    H = np.stack([ctx.colloid_force_history(0, k, steps) for k in range(n)], axis=1)   # steps x n x 12
    return dict(ctx=ctx, ref=ref, Q=ctx.get_Q(0), f=ctx.get_f(0), u=ctx.get_u(0), Qr=ref.get_Q(), fr=ref.get_f(),
                ur=ref.get_u(), fluid=~ref.solid(), H=H, Hr=np.array(hist))


def check_multi(r, tol_q, tol_f, tol_force, tol_u=None):
    m = r["fluid"]
    eq = max(rel_inf(r["Q"], r["Qr"], m), rel_l2(r["Q"], r["Qr"], m))
    ef = max(rel_inf(r["f"], r["fr"], m), rel_l2(r["f"], r["fr"], m))
    say("   rel err Q %.3e f %.3e" % (eq, ef))
    assert eq < tol_q and ef < tol_f
    if tol_u is not None:
        eu = rel_inf(r["u"], r["ur"], m)
        say("   rel err u %.3e" % eu)
        assert eu < tol_u
    for k in range(r["H"].shape[1]):
        F, Fr = r["H"][:, k], r["Hr"][:, k]
        err = np.linalg.norm(F - Fr)
        bound = max(tol_force * np.linalg.norm(Fr), 1e-6 * math.sqrt(F.shape[0]))
        say("   colloid %d force err %.3e bound %.3e (|F| %.3e)" % (k, err, bound, np.linalg.norm(Fr)))
        assert err <= bound
    pos = np.array([list(c.pos) for c in r["ctx"].get_colloids(0)])
    pos_r = np.array([list(c.pos) for c in r["ref"].get_colloids()])
    np.testing.assert_allclose(pos, pos_r, rtol=0, atol=1e-9)


TWO_FIXED = [dict(pos=(6.3, 7.1, 5.8), a0=3.2, anchoring="planar", W=0.02, S0=0.5),
             dict(pos=(16.6, 15.2, 17.4), a0=4.4, anchoring="normal", W=math.inf, S0=0.5)]
THREE_MOVING = [dict(pos=(6.3, 7.1, 5.8), a0=3.2, anchoring="planar", W=0.02, S0=0.5, vel=(0.05, 0.0, -0.03),
                     omega=(0.0, 0.004, 0.0), motion=1),
                dict(pos=(16.6, 15.2, 17.4), a0=4.4, anchoring="normal", W=math.inf, S0=0.5, vel=(-0.02, 0.04, 0.0),
                     omega=(0.003, 0.0, 0.0), motion=1),
                dict(pos=(5.5, 18.3, 16.9), a0=2.7, anchoring="normal", W=0.05, S0=0.5)]
TWO_FREE = [dict(pos=(6.3, 7.1, 5.8), a0=3.2, anchoring="planar", W=0.02, S0=0.5, motion=2, vel=(0.02, 0.0, -0.01),
                 fext=(1e-3, 0.0, 5e-4), rho_c=1.2),
            dict(pos=(16.6, 15.2, 17.4), a0=4.4, anchoring="normal", W=0.01, S0=0.5, motion=2, vel=(-0.01, 0.02, 0.0),
                 omega=(0.0, 0.0, 0.002), rho_c=0.9)]


@pytest.mark.parametrize("name,specs", [("two fixed", TWO_FIXED), ("three prescribed/fixed", THREE_MOVING),
                                        ("two free", TWO_FREE)])
def test_fp64_colloids_against_oracle(name, specs):
    say("case: 24^3 fp64 chiral, %s, 30 steps" % name)
    L = 24
    prm = dict(NEM, q0=0.15)
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=101, noise=0.02, director=(1, 0.3, 0.6))
    r = run_multi(L, prm, 30, "fp64", specs, Q0)
    check_multi(r, 1e-10, 1e-12, 1e-8, tol_u=1e-8)
    if name == "two free":
        v = np.array([list(c.vel) + list(c.omega) for c in r["ctx"].get_colloids(0)])
        vr = np.array([list(c.vel) + list(c.omega) for c in r["ref"].get_colloids()])
        np.testing.assert_allclose(v, vr, rtol=1e-9, atol=1e-13)


def test_fp64_colloids_with_variants():
    say("case: 24^3 fp64 third-order advection and 27-point stencil, three colloids, 25 steps")
    L = 24
    prm = dict(NEM, q0=0.15, advection=3, stencil=27)
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=102, noise=0.02, director=(1, 0.3, 0.6))
    r = run_multi(L, prm, 25, "fp64", THREE_MOVING, Q0)
    check_multi(r, 1e-10, 1e-12, 1e-8, tol_u=1e-8)


def test_fp32_colloids_against_oracle():
    say("case: 48^3 fp32 cholesteric, three colloids (two moving), 60 steps")
    L = 48
    q0 = 2 * math.pi / 24
    prm = dict(NEM, q0=q0)
    specs = [dict(pos=(12.3, 13.1, 11.8), a0=6.2, anchoring="normal", W=math.inf, S0=0.5, vel=(0.03, 0.0, -0.01),
                  motion=1),
             dict(pos=(34.6, 33.2, 35.4), a0=7.4, anchoring="planar", W=0.02, S0=0.5),
             dict(pos=(11.5, 36.3, 34.9), a0=5.7, anchoring="normal", W=0.05, S0=0.5, vel=(0.0, -0.02, 0.02),
                  omega=(0.0, 0.0, 0.003), motion=1)]
    r = run_multi(L, prm, 60, "fp32", specs, inputs.helix_q(L, L, L, q0, inputs.Q_INIT))
    check_multi(r, 1e-5, 1e-5, 1e-3)


def test_solid_map_from_the_library():
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: library solid map, three colloids on 24^3")
    L = 24
    ctx = lc.Context([dict(nx=L, precision="fp32", **NEM)])
    ctx.set_colloids(0, THREE_MOVING)
    ref = lco.Sim(L, **NEM)
    ref.set_colloids(_oracle_specs(THREE_MOVING))
    np.testing.assert_array_equal(ctx.solid_id(0), ref.solid_id())
    ctx.step(7)
    ref.step(7)
    np.testing.assert_array_equal(ctx.solid_id(0), ref.solid_id())
    ctx.close()


def test_colloids_closer_than_the_gap():
    from paper_1102_2193_amd import lc
    say("case: separation rule on 24^3")
    L = 24
    ctx = lc.Context([dict(nx=L, precision="fp64", **NEM)])
    with pytest.raises(lc.LCError) as e:
        ctx.set_colloids(0, [dict(pos=(8.0, 8.0, 8.0), a0=3.0), dict(pos=(16.5, 8.0, 8.0), a0=3.0)])
    assert e.value.code == 1
    assert ctx.num_colloids(0) == 0
    ctx.set_colloids(0, [dict(pos=(8.0, 8.0, 8.0), a0=3.0, vel=(0.25, 0, 0), motion=1),
                         dict(pos=(17.2, 8.0, 8.0), a0=3.0)])
    ctx.step(1)                 # starts 3.2 apart
    ctx.sync()
    ctx.step(1)                 # starts 2.95 apart
    with pytest.raises(lc.LCError) as e:
        ctx.sync()
    assert e.value.code == 5
    ctx.close()


def test_checkpoint_with_colloids_continues_bit_for_bit():
    from paper_1102_2193_amd import lc
    say("case: checkpoint of a box with three colloids")
    L = 24
    prm = dict(nx=L, precision="fp32", **dict(NEM, q0=0.15))
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=103, noise=0.02)
    a = lc.Context([prm])
    a.set_colloids(0, THREE_MOVING)
    a.set_Q(0, Q0)
    a.step(9)
    state = a.get_state()
    a.step(21)
    b = lc.Context([prm])
    b.set_state(state)
    assert b.num_colloids(0) == 3
    b.step(21)
    for k in range(3):
        np.testing.assert_array_equal(a.colloid_force_history(0, k, 30), b.colloid_force_history(0, k, 30))
    np.testing.assert_array_equal(a.get_Q(0), b.get_Q(0))
    np.testing.assert_array_equal(a.get_f(0), b.get_f(0))
    a.close()
    b.close()


def test_batch_boxes_with_different_colloid_counts():
    """A batch whose boxes hold 0, 1 and 3 colloids matches each box run
    alone; setting the colloids of one box later keeps the other boxes'
    force histories."""
    from paper_1102_2193_amd import lc
    say("case: batch of boxes with 0, 1 and 3 colloids")
    boxes = [dict(nx=24, precision="fp32", **NEM), dict(nx=20, precision="fp32", **dict(NEM, q0=0.2)),
             dict(nx=24, precision="fp32", **dict(NEM, q0=0.15))]
    cols = [[], [dict(pos=(10.2, 9.7, 10.4), a0=4.0, anchoring="planar", W=0.02)], THREE_MOVING]
    Qs = [inputs.noisy_nematic_q(b["nx"], b["nx"], b["nx"], inputs.Q_INIT, seed=110 + i, noise=0.02)
          for i, b in enumerate(boxes)]
    ctx = lc.Context(boxes)
    for b, cl in enumerate(cols):
        ctx.set_colloids(b, cl)
        ctx.set_Q(b, Qs[b])
    assert tuple(ctx.tile_shape(ctx.get_tile())) == (16, 8, 2)
    ctx.step(12)
    h1 = ctx.colloid_force_history(1, 0, 12)
    for b, cl in enumerate(cols):
        single = lc.Context([boxes[b]])
        single.set_colloids(0, cl)
        # the batch runs on the 3D tile (one of its boxes holds three colloids)
        single.set_tile(ctx.get_tile())
        single.set_Q(0, Qs[b])
        single.step(12)
        np.testing.assert_array_equal(ctx.get_Q(b), single.get_Q(0))
        np.testing.assert_array_equal(ctx.get_f(b), single.get_f(0))
        for k in range(len(cl)):
            np.testing.assert_array_equal(ctx.colloid_force_history(b, k, 12), single.colloid_force_history(0, k, 12))
        single.close()
    # box 0 gains two colloids: box 1 keeps its history
    ctx.set_colloids(0, TWO_FIXED)
    np.testing.assert_array_equal(ctx.colloid_force_history(1, 0, 12), h1)
    ctx.step(3)
    assert np.all(np.isfinite(ctx.colloid_force_history(0, 1, 3)))
    ctx.close()
