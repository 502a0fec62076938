"""GPU parity outside the unit-relaxation regime and at the workloads' full sizes.

* The paper's material parameters (Sec. 2.1: A0 = 1, K = 0.065, gamma = 3,
  xi = 0.7, Gamma = 0.5) with BGK relaxation times tau = 0.8 (the
  viscosity 0.1 of Sec. 3.1) and tau = 1.5.  At tau = 1 the collision
  forgets f (f* = f_eq + S/2), so only tau != 1 exercises the relaxation
  term and the Guo source factor 1 - 1/(2 tau).  Planar anchoring (the
  paper's fixed Q^0), a fixed and a free colloid.  FP64 to round-off; FP32
  to 1e-5 on Q and f, 1e-3 on the force, and element by element on the
  deviations from rest f - w and on u (bound below).
* The 128^3 drag workload for 100 steps (along x on every tile, along z on
  the default one), the 128^3 cholesteric workload
  with the a = 16 colloid, the 256^3 nematic workload, and the 48-box batch
  against one oracle run per box; the largest box the marching kernel takes.

FP32 bound on f - w and u, element by element relative to the largest
reference value over fluid sites: each step rounds u = (j + F/2)/rho and
the populations it forms to FP32 (relative 2^-24 of rho ~ 1 and of the
force sums), and these errors add over the steps at most linearly, so
after n steps the deviation is below c n 2^-24 relative to the largest
value; c = 40 covers the force term, whose face differences cancel digits
of the stress (measured: well inside it, see the printed errors).
"""
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs
from test_parity_gpu import ANCH, check, rel_inf, rel_l2, run_pair, say

pytestmark = pytest.mark.gpu

PAPER = dict(inputs.PAPER_CHOLESTERIC)
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def fp32_dev_bound(nsteps):
    return 40.0 * nsteps * 2.0 ** -24


def check_dev(r, bound):
    """f - w and u element by element over fluid sites."""
    m = r["fluid"]
    fw, fwr = r["f"] - W19[:, None, None, None], r["fr"] - W19[:, None, None, None]
    ef = rel_inf(fw, fwr, m)
    eu = rel_inf(r["u"], r["ur"], m)
    say("   rel err f - w %.3e, u %.3e (bound %.3e)" % (ef, eu, bound))
    assert ef < bound, ("f - w", ef, bound)
    assert eu < bound, ("u", eu, bound)


def planar_colloid(pos, a0, motion):
    c = dict(pos=pos, a0=a0, anchoring="planar", W=math.inf, S0=0.5)
    if motion == "free":
        c.update(motion=2, vel=(0.01, 0.0, -0.005), omega=(0.0, 0.001, 0.0), fext=(0.02, 0.0, -0.01), rho_c=1.0)
    return c


@pytest.mark.parametrize("tau", [0.8, 1.5])
@pytest.mark.parametrize("motion", ["fixed", "free"])
def test_fp64_paper_parameters_tau(tau, motion):
    say("case: 16^3 fp64 A0=1 K=0.065 tau=%g planar W=inf, %s colloid a=4, 40 steps" % (tau, motion))
    L = 16
    prm = dict(PAPER, tau=tau)
    Q0 = inputs.noisy_nematic_q(L, L, L, 0.5, seed=51, noise=0.02, director=(1, 0.2, 0.4))
    r = run_pair((L, L, L), prm, 40, "fp64", colloid=planar_colloid((7.6, 8.3, 8.1), 4.0, motion), Q0=Q0,
                 hist=True)
    check(r, 1e-10, 1e-12, tol_u=1e-8, tol_force=1e-8)
    check_dev(r, 1e-9)
    if motion == "free":
        c, oc = r["ctx"].get_colloid(0), r["ref"].get_colloid()
        np.testing.assert_allclose(np.array(list(c.pos) + list(c.vel)), np.array(list(oc.pos) + list(oc.vel)),
                                   rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("tau", [0.8, 1.5])
@pytest.mark.parametrize("motion", ["fixed", "free"])
def test_fp32_paper_parameters_tau(tau, motion):
    say("case: 32^3 fp32 A0=1 K=0.065 tau=%g planar W=inf, %s colloid a=6, 100 steps" % (tau, motion))
    L, n = 32, 100
    prm = dict(PAPER, tau=tau)
    Q0 = inputs.noisy_nematic_q(L, L, L, 0.5, seed=52)
    r = run_pair((L, L, L), prm, n, "fp32", colloid=planar_colloid((15.6, 16.3, 16.2), 6.0, motion), Q0=Q0,
                 hist=True)
    check(r, 1e-5, 1e-5, tol_force=1e-3)
    check_dev(r, fp32_dev_bound(n))
    d = r["ctx"].diag(0)
    say("   max |u| %.3e" % d["umax"])
    assert d["umax"] > 1e-5   # the anchoring drives a flow: the relaxation term is exercised


def test_full_size_drag128_100_steps_every_tile():
    """The benchmark's workload (128^3 FP32, a = 8 moving along x, normal
    anchoring W = 0.01) with graph replay, the benchmark's stepping, for 100
    steps against one oracle run, for every FP32 tile shape (the benchmark
    times the one its tuner picks)."""
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: 128^3 fp32 drag workload, 100 steps vs oracle, every tile")
    L, n = 128, 100
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=2)
    col = dict(pos=(64.0, 64.0, 64.0), a0=8.0, anchoring="normal", W=0.01, S0=0.5, vel=(1e-3, 0, 0))
    ref = lco.Sim(L, **inputs.NEMATIC)
    ref.set_colloid(col["pos"], col["a0"], anchoring=ANCH["normal"], W=0.01, S0=0.5, vel=col["vel"],
                    motion=lco.PRESCRIBED)
    ref.set_Q(Q0)
    hr = []
    for _ in range(n):
        ref.step(1)
        hr.append(ref.force())
    base = dict(Qr=ref.get_Q(), fr=ref.get_f(), ur=ref.get_u(), Hr=np.array(hr), fluid=~ref.solid())
    pos_ref = np.array(ref.get_colloid().pos)
    ntile = None
    t = 0
    while ntile is None or t < ntile:
        ctx = lc.Context([dict(nx=L, precision="fp32", **inputs.NEMATIC)])
        ntile = ctx.num_tiles()
        ctx.set_tile(t)
        ctx.set_colloid(0, col["pos"], col["a0"], anchoring="normal", W=0.01, S0=0.5, vel=col["vel"],
                        motion=lc.PRESCRIBED)
        ctx.set_Q(0, Q0)
        ctx.step(n)
        say("  tile %d %s" % (t, ctx.tile_shape(t)))
        r = dict(base, Q=ctx.get_Q(0), f=ctx.get_f(0), u=ctx.get_u(0), H=ctx.force_history(0, n))
        check(r, 1e-5, 1e-5, tol_force=1e-3)
        check_dev(r, fp32_dev_bound(n))
        np.testing.assert_array_equal(np.array(ctx.get_colloid(0).pos), pos_ref)
        ctx.close()
        t += 1


def test_full_size_drag128_along_z():
    """The drag workload's second leg: the same colloid dragged along z, the
    direction the marching kernel sweeps its planes, so the planes with
    solid nodes move through the planned work items; the default tile and
    graph replay, 100 steps against one oracle run."""
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: 128^3 fp32 drag workload along z, 100 steps vs oracle")
    L, n = 128, 100
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=2)
    col = dict(pos=(64.0, 64.0, 64.0), a0=8.0, anchoring="normal", W=0.01, S0=0.5, vel=(0, 0, 1e-3))
    ref = lco.Sim(L, **inputs.NEMATIC)
    ref.set_colloid(col["pos"], col["a0"], anchoring=ANCH["normal"], W=0.01, S0=0.5, vel=col["vel"],
                    motion=lco.PRESCRIBED)
    ref.set_Q(Q0)
    hr = []
    for _ in range(n):
        ref.step(1)
        hr.append(ref.force())
    ctx = lc.Context([dict(nx=L, precision="fp32", **inputs.NEMATIC)])
    ctx.set_colloid(0, col["pos"], col["a0"], anchoring="normal", W=0.01, S0=0.5, vel=col["vel"],
                    motion=lc.PRESCRIBED)
    ctx.set_Q(0, Q0)
    ctx.step(n)
    say("  tile %s" % (ctx.tile_shape(ctx.get_tile()),))
    r = dict(Q=ctx.get_Q(0), f=ctx.get_f(0), u=ctx.get_u(0), H=ctx.force_history(0, n), Qr=ref.get_Q(),
             fr=ref.get_f(), ur=ref.get_u(), Hr=np.array(hr), fluid=~ref.solid())
    check(r, 1e-5, 1e-5, tol_force=1e-3)
    check_dev(r, fp32_dev_bound(n))
    np.testing.assert_array_equal(np.array(ctx.get_colloid(0).pos), np.array(ref.get_colloid().pos))
    ctx.close()


def test_full_size_cholesteric128_a16():
    say("case: 128^3 fp32 cholesteric p=32, fixed homeotropic a=16 W=inf, 20 steps vs oracle")
    L, n = 128, 20
    q0 = 2 * math.pi / 32
    prm = dict(inputs.NEMATIC, q0=q0)
    col = dict(pos=(64.0, 64.0, 64.0), a0=16.0, anchoring="normal", W=math.inf, S0=0.5)
    Q0 = inputs.helix_q(L, L, L, q0, inputs.Q_INIT)
    r = run_pair((L, L, L), prm, n, "fp32", colloid=col, Q0=Q0, hist=True)
    check(r, 1e-5, 1e-5, tol_force=1e-3)
    check_dev(r, fp32_dev_bound(n))


def test_full_size_nematic256():
    """The 256^3 workload (nematic, a = 16 normal colloid with W = 0.01 at the
    centre, the benchmark's inputs) on the 64 x 8 marching tile the tuner
    picks at this size and on the default 32 x 16, 10 steps against one
    oracle run."""
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: 256^3 fp32 nematic workload, a = 16, 10 steps vs oracle, tiles 64x8 and 32x16")
    L, n = 256, 10
    c = (L / 2,) * 3
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=2)
    ref = lco.Sim(L, **inputs.NEMATIC)
    ref.set_colloid(c, 16.0, anchoring=ANCH["normal"], W=0.01, S0=0.5)
    ref.set_Q(Q0)
    hr = []
    for _ in range(n):
        ref.step(1)
        hr.append(ref.force())
    base = dict(Qr=ref.get_Q(), fr=ref.get_f(), ur=ref.get_u(), Hr=np.array(hr), fluid=~ref.solid())
    del ref
    say("   oracle done")
    for shape in ((64, 8, 8), (32, 16, 8)):
        ctx = lc.Context([dict(nx=L, precision="fp32", **inputs.NEMATIC)])
        ctx.set_tile([t for t in range(ctx.num_tiles()) if tuple(ctx.tile_shape(t)) == shape][0])
        ctx.set_colloid(0, c, 16.0, anchoring="normal", W=0.01, S0=0.5)
        ctx.set_Q(0, Q0)
        ctx.step(n)
        say("  tile %s" % (shape,))
        r = dict(base, Q=ctx.get_Q(0), f=ctx.get_f(0), u=ctx.get_u(0), H=ctx.force_history(0, n))
        check(r, 1e-5, 1e-5, tol_force=1e-3)
        check_dev(r, fp32_dev_bound(n))
        ctx.close()


def test_batch48_against_oracle_per_box():
    """The 48-box batch (L in {32..64}, a in [3, 12], pitch in [16, 48]
    commensurate, fixed homeotropic colloids) in one context for 20 steps,
    each box against its own oracle run; the default marching tile, the
    wide one and the 3D tile (the shapes the tuner chooses among for it)."""
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: batch of 48 cholesteric fp32 boxes, 20 steps vs one oracle run per box")
    n = 20
    specs = inputs.batch_boxes(4)
    boxes = [dict(nx=s["L"], precision="fp32", **dict(inputs.NEMATIC, q0=s["q0"])) for s in specs]
    Qs = [inputs.helix_q(s["L"], s["L"], s["L"], s["q0"], inputs.Q_INIT) for s in specs]
    refs = []
    for b, s in enumerate(specs):
        L, c = s["L"], s["L"] / 2.0
        ref = lco.Sim(L, **dict(inputs.NEMATIC, q0=s["q0"]))
        ref.set_colloid((c, c, c), s["a"], anchoring=ANCH["normal"], W=math.inf)
        ref.set_Q(Qs[b])
        hr = []
        for _ in range(n):
            ref.step(1)
            hr.append(ref.force())
        refs.append((ref.get_Q(), ref.get_f(), np.array(hr), ~ref.solid()))
        del ref
    say("   oracle done: %d sites" % sum(s["L"] ** 3 for s in specs))
    for shape in ((32, 16, 8), (64, 8, 8), (16, 8, 2)):
        ctx = lc.Context(boxes)
        tile = [t for t in range(ctx.num_tiles()) if tuple(ctx.tile_shape(t)) == shape][0]
        ctx.set_tile(tile)
        for b, s in enumerate(specs):
            c = s["L"] / 2.0
            ctx.set_colloid(b, (c, c, c), s["a"], anchoring="normal", W=math.inf)
            ctx.set_Q(b, Qs[b])
        ctx.step(n)
        worst = 0.0
        for b, (Qr, fr, Hr, m) in enumerate(refs):
            Q, f = ctx.get_Q(b), ctx.get_f(b)
            eq = max(rel_inf(Q, Qr, m), rel_l2(Q, Qr, m))
            ef = max(rel_inf(f, fr, m), rel_l2(f, fr, m))
            eF = np.linalg.norm(ctx.force_history(b, n) - Hr)
            bound = max(1e-3 * np.linalg.norm(Hr), 1e-6 * math.sqrt(n))
            worst = max(worst, eq, ef)
            assert eq < 1e-5 and ef < 1e-5, (shape, b, eq, ef)
            assert eF <= bound, (shape, b, eF, bound)
        say("   tile %s: worst rel err of Q and f over the 48 boxes %.3e" % (shape, worst))
        ctx.close()


def _tiled_equal(big, small, rx, ry):
    """big (nc, nz, ry ny, rx nx) equals small (nc, nz, ny, nx) repeated
    rx times in x and ry times in y, bit for bit (plane chunk by chunk)."""
    nc, nz, sy, sx = small.shape
    b = big.reshape(nc, nz, ry, sy, rx, sx)
    c = small.reshape(nc, nz, 1, sy, 1, sx)
    return all(bool(np.array_equal(b[:, z0:z0 + 16], np.broadcast_to(c[:, z0:z0 + 16], b[:, z0:z0 + 16].shape)))
               for z0 in range(0, nz, 16))


def test_largest_marching_box_against_a_repeated_cell():
    """The largest FP32 box the marching kernel takes: 384 x 384 x 383 sites,
    whose 19 population components span 4,292,149,248 bytes, just under the
    4 GiB that the kernel's 32-bit component offsets reach; one plane more
    and the library refuses the marching shapes and defaults to the 3D tile.
    The initial Q repeats with period 8 in x and y and there is no colloid,
    so every site of the box must evolve as the same site of a 32 x 16 x 383
    box with the same repeated start, on the same marching shape: Q, f and u
    bit for bit (each site's arithmetic does not depend on how the planes
    are split into work items), and that box against one oracle run of the
    8 x 8 x 383 cell (the paper's parameters with pitch 32, tau = 0.8,
    20 steps; Q and f to 1e-5, u to the bound below)."""
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: 384x384x383 fp32 (marching kernel at its 4 GiB offset limit), 20 steps vs 32x16x383 and an 8x8x383 oracle cell")
    C, NZ, n = 8, 383, 20
    prm = dict(PAPER, tau=0.8, q0=2 * math.pi / 32)
    Qc = inputs.noisy_nematic_q(C, C, NZ, 0.5, seed=57, noise=0.02, director=(1, 0.2, 0.4))
    ref = lco.Sim(C, C, NZ, **prm)
    ref.set_Q(Qc)
    ref.step(n)
    cell = dict(Q=ref.get_Q(), f=ref.get_f(), u=ref.get_u())
    del ref
    ctx = lc.Context([dict(nx=32, ny=16, nz=NZ, precision="fp32", **prm)])
    ctx.set_tile([t for t in range(ctx.num_tiles()) if tuple(ctx.tile_shape(t)) == (32, 16, 8)][0])
    ctx.set_Q(0, np.tile(Qc, (1, 1, 2, 4)))
    ctx.step(n)
    small = dict(Q=ctx.get_Q(0), f=ctx.get_f(0), u=ctx.get_u(0))
    ctx.close()
    # u: each step's force density is a difference of FP32 stresses of size
    # up to A0 S^2 = 0.25, rounded to 2^-24 relative, so after n steps u is
    # off by at most about n 2^-24 0.25 in absolute terms
    fluid = np.ones((NZ, 16, 32), dtype=bool)
    umax = np.max(np.abs(cell["u"]))
    for k, tol in (("Q", 1e-5), ("f", 1e-5), ("u", n * 2.0 ** -24 * 0.25 / umax)):
        ref_k = np.tile(cell[k], (1, 1, 2, 4))
        e = max(rel_inf(small[k], ref_k, fluid), rel_l2(small[k], ref_k, fluid))
        say("   32x16x383 vs oracle: rel err %s %.3e (bound %.3e)" % (k, e, tol))
        assert e < tol, (k, e)
    assert umax > 1e-4   # the tilt and the noise drive a flow
    L = 384
    assert 19 * 4 * L * L * NZ < 2 ** 32 <= 19 * 4 * L * L * (NZ + 1)
    ctx = lc.Context([dict(nx=L, ny=L, nz=NZ, precision="fp32", **prm)])
    shape = ctx.tile_shape(ctx.get_tile())
    nblk, _ = ctx.launch_info()
    say("   default tile %s, %d blocks" % (shape, nblk))
    assert tuple(shape) == (32, 16, 8)   # the marching kernel's default shape
    ctx.set_Q(0, np.tile(Qc, (1, 1, L // C, L // C)))
    ctx.step(n)
    for k, get in (("Q", ctx.get_Q), ("f", ctx.get_f), ("u", ctx.get_u)):
        same = _tiled_equal(get(0), small[k], L // 32, L // 16)
        say("   384x384x383 %s equal to the repeated 32x16x383 box: %s" % (k, same))
        assert same, k
    ctx.close()
    # one plane more: 19 x 4 x sites reaches 4 GiB
    ctx = lc.Context([dict(nx=L, ny=L, nz=NZ + 1, precision="fp32", **prm)])
    assert tuple(ctx.tile_shape(ctx.get_tile())) == (16, 8, 2)
    march = [t for t in range(ctx.num_tiles()) if tuple(ctx.tile_shape(t)) == (32, 16, 8)][0]
    with pytest.raises(lc.LCError, match="too large for the marching kernel"):
        ctx.set_tile(march)
    ctx.close()
