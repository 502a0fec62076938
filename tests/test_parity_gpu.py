"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars (checked element by element over fluid sites):
  FP64 library vs oracle: round-off (relative 1e-10 on Q, f and u).
  FP32 library vs oracle: 1e-5 relative on Q and f, 1e-3 on the colloid force.
Every case prints its name before touching the GPU.
"""
import math
import sys

import numpy as np
import pytest

from paper_1102_2193_amd import inputs

pytestmark = pytest.mark.gpu

NEM = inputs.NEMATIC
ANCH = {"none": 0, "normal": 1, "planar": 2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_inf(a, b, mask):
    d = np.max(np.abs(a - b)[:, mask])
    return d / max(np.max(np.abs(b[:, mask])), 1e-300)


def rel_l2(a, b, mask):
    d = np.linalg.norm((a - b)[:, mask])
    return d / max(np.linalg.norm(b[:, mask]), 1e-300)


def run_pair(dims, prm, steps, precision, colloid=None, Q0=None, tile=None, graph=True, f0=None,
             hist=False):
    """Run the same seeded case on the GPU and on the oracle."""
    from oracle import lco
    from paper_1102_2193_amd import lc
    nx, ny, nz = dims
    ctx = lc.Context([dict(nx=nx, ny=ny, nz=nz, precision=precision, **prm)])
    if tile is not None:
        ctx.set_tile(tile)
    ctx.use_graph(graph)
    ref = lco.Sim(nx, ny, nz, **{k: v for k, v in prm.items()})
    if colloid is not None:
        c = dict(colloid)
        pos, a0 = c.pop("pos"), c.pop("a0")
        ctx.set_colloid(0, pos, a0, **c)
        oc = dict(c)
        oc["anchoring"] = ANCH[oc.get("anchoring", "normal")] if isinstance(oc.get("anchoring", "normal"), str) \
            else oc["anchoring"]
        ref.set_colloid(pos, a0, **oc)
    if Q0 is not None:
        ctx.set_Q(0, Q0)
        ref.set_Q(Q0)
    if f0 is not None:
        ctx.set_f(0, f0)
        ref.set_f(f0)
    ctx.step(steps)
    ref_hist = []
    if hist:
        for _ in range(steps):
            ref.step(1)
            ref_hist.append(ref.force())
    else:
        ref.step(steps)
    out = dict(Q=ctx.get_Q(0), f=ctx.get_f(0), u=ctx.get_u(0), F=ctx.force(0),
               Qr=ref.get_Q(), fr=ref.get_f(), ur=ref.get_u(), Fr=ref.force(), fluid=~ref.solid(),
               ctx=ctx, ref=ref)
    if hist:
        out["H"] = ctx.force_history(0, steps)
        out["Hr"] = np.array(ref_hist)
    return out


def check(r, tol_q, tol_f, tol_u=None, tol_force=None):
    """tol_f None: the fluid is off (hydro = 0) and f is not part of the state."""
    m = r["fluid"]
    eq = max(rel_inf(r["Q"], r["Qr"], m), rel_l2(r["Q"], r["Qr"], m))
    say("   rel err Q %.3e" % eq)
    assert eq < tol_q, ("Q", eq)
    if tol_f is not None:
        ef = max(rel_inf(r["f"], r["fr"], m), rel_l2(r["f"], r["fr"], m))
        say("   rel err f %.3e" % ef)
        assert ef < tol_f, ("f", ef)
    if tol_u is not None:
        eu = rel_inf(r["u"], r["ur"], m)
        say("   rel err u %.3e" % eu)
        assert eu < tol_u, ("u", eu)
    if tol_force is not None:
        if "H" in r:
            F, Fr = r["H"], r["Hr"]
        else:
            F, Fr = r["F"][None], r["Fr"][None]
        # A force that vanishes by symmetry leaves only the effect of the FP32
        # field error (~1e-9 per population, coherent over thousands of
        # links: ~1e-7 per step): absolute floor of 1e-6 per step.
        err = np.linalg.norm(F - Fr)
        bound = max(tol_force * np.linalg.norm(Fr), 1e-6 * math.sqrt(F.shape[0]))
        say("   force err %.3e bound %.3e (|F| %.3e)" % (err, bound, np.linalg.norm(Fr)))
        assert err <= bound, ("force", err, bound)


CFG0 = dict(pos=(16.0, 16.0, 16.0), a0=4.0, anchoring="planar", W=0.01, S0=0.5)


def test_fp64_parity_nematic32_planar():
    say("case: 32^3 fp64 planar W=0.01 a=4, 200 steps")
    L = 32
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=1)
    r = run_pair((L, L, L), NEM, 200, "fp64", colloid=CFG0, Q0=Q0, hist=True)
    check(r, 1e-10, 1e-12, tol_u=1e-8, tol_force=1e-8)
    # deviations from rest carry the dynamics: compare them too
    m = r["fluid"]
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]
    dev = rel_inf(r["f"][:, m] - w, r["fr"][:, m] - w, np.ones(m.sum(), bool))
    say("   rel err f - w %.3e" % dev)
    assert dev < 1e-9


def test_fp32_parity_nematic32_planar():
    say("case: 32^3 fp32 planar W=0.01 a=4, 100 steps")
    L = 32
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=1)
    r = run_pair((L, L, L), NEM, 100, "fp32", colloid=CFG0, Q0=Q0, hist=True)
    check(r, 1e-5, 1e-5, tol_force=1e-3)


def test_fp32_colloid_moving_past_the_planned_split():
    # The marching kernel's work split is planned on the host from the
    # colloid position at set-up (two sites of slack); the kernels test the
    # live position, so a colloid that travels further still gets the
    # solid-aware path wherever it reaches.
    say("case: 32^3 fp32 cholesteric, colloid moving 4.8 sites in 60 steps")
    L = 32
    prm = dict(NEM, q0=2 * math.pi / 16)
    Q0 = inputs.helix_q(L, L, L, 2 * math.pi / 16, inputs.Q_INIT)
    col = dict(pos=(9.3, 16.2, 15.7), a0=4.0, anchoring="normal", W=0.02, S0=0.5, vel=(0.08, 0.01, -0.02),
               motion=1)
    r = run_pair((L, L, L), prm, 60, "fp32", colloid=col, Q0=Q0, hist=True)
    check(r, 1e-5, 1e-5, tol_force=1e-3)
    np.testing.assert_array_equal(np.array(r["ctx"].get_colloid(0).pos), np.array(r["ref"].get_colloid().pos))


MODES = [(anch, motion, hydro) for anch in ("none", "normal", "planar") for motion in (0, 1) for hydro in (0, 1)]


@pytest.mark.parametrize("anch,motion,hydro", MODES)
def test_fp64_brute_force_modes(anch, motion, hydro):
    say("case: 12^3 fp64 anchoring=%s motion=%d hydro=%d" % (anch, motion, hydro))
    L = 12
    prm = dict(NEM, hydro=hydro, q0=0.2)
    col = dict(pos=(6.3, 5.8, 6.1), a0=3.1, anchoring=anch, W=0.02 if anch != "normal" else math.inf,
               S0=0.5, vel=(0.04, -0.02, 0.03) if motion else (0, 0, 0), omega=(0.0, 0.0, 0.002),
               motion=motion)
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=21, noise=0.02, director=(1, 0.2, 0.4))
    r = run_pair((L, L, L), prm, 30, "fp64", colloid=col, Q0=Q0, hist=True)
    assert np.all(np.isfinite(r["Q"]))
    check(r, 1e-10, 1e-12 if hydro else None, tol_u=1e-8 if hydro else None,
          tol_force=1e-8 if hydro else None)
    if motion:
        c = r["ctx"].get_colloid(0)
        oc = r["ref"].get_colloid()
        np.testing.assert_array_equal(np.array(c.pos), np.array(oc.pos))


@pytest.mark.parametrize("tile", [0, 1])
def test_fp64_ragged_box_every_tile(tile):
    say("case: 20x12x10 fp64 tile %d" % tile)
    dims = (20, 12, 10)
    prm = dict(NEM, q0=0.15)
    col = dict(pos=(9.5, 6.2, 5.0), a0=2.6, anchoring="normal", W=0.05, S0=0.45)
    Q0 = inputs.noisy_nematic_q(*dims, inputs.Q_INIT, seed=5, noise=0.01)
    r = run_pair(dims, prm, 25, "fp64", colloid=col, Q0=Q0, tile=tile, hist=True)
    check(r, 1e-10, 1e-12, tol_u=1e-8, tol_force=1e-8)


def test_fp32_tiles_agree():
    from paper_1102_2193_amd import lc
    say("case: 40x24x16 fp32, all tiles")
    dims = (40, 24, 16)
    Q0 = inputs.noisy_nematic_q(*dims, inputs.Q_INIT, seed=6)
    res = []
    ntile = None
    for tile in range(64):
        ctx = lc.Context([dict(nx=dims[0], ny=dims[1], nz=dims[2], precision="fp32", **NEM)])
        ntile = ctx.num_tiles()
        if tile >= ntile:
            break
        ctx.set_tile(tile)
        ctx.set_colloid(0, (20.0, 12.0, 8.0), 5.0, anchoring="planar", W=0.01)
        ctx.set_Q(0, Q0)
        ctx.step(20)
        res.append((ctx.tile_shape(tile), ctx.get_Q(0), ctx.get_f(0), ctx.force(0)))
        ctx.close()
    for shape, Q, f, F in res[1:]:
        dq = np.max(np.abs(Q - res[0][1]))
        df = np.max(np.abs(f - res[0][2]))
        say("   tile %s: max |dQ| %.3e |df| %.3e" % (shape, dq, df))
        assert dq < 1e-6 and df < 1e-7
        # tile shapes change only the rounding of the stress (FP32 ulps)
        assert np.linalg.norm(F - res[0][3]) <= 1e-4 * np.linalg.norm(res[0][3]) + 1e-8


def test_march_blocks_with_several_items_agree_with_3d_tiles():
    """512 x 512 x 16: the 32x16 and 64x8 column tiles give 512 column
    blocks, more than the resident blocks of the persistent kernel, so every
    block marches two or more work items (the layout of large boxes); the
    3D-tile kernel, which has no schedule, is the reference."""
    from paper_1102_2193_amd import lc
    say("case: 512x512x16 fp32, marching tiles with several items per block vs the 3D tile")
    dims = (512, 512, 16)
    Q0 = inputs.noisy_nematic_q(*dims, inputs.Q_INIT, seed=7)
    res = {}
    for tile in (6, 5, 8):
        ctx = lc.Context([dict(nx=dims[0], ny=dims[1], nz=dims[2], precision="fp32", **NEM)])
        shape = ctx.tile_shape(tile)
        ctx.set_tile(tile)
        nblk, _ = ctx.launch_info()
        if tile != 6:
            ncb = (dims[0] // shape[0]) * (dims[1] // shape[1])
            say("   tile %s: %d column blocks on %d blocks" % (shape, ncb, nblk))
            assert ncb > nblk
        ctx.set_colloid(0, (256.0, 256.0, 8.0), 5.0, anchoring="normal", W=0.01)
        ctx.set_Q(0, Q0)
        ctx.step(10)
        res[tile] = (ctx.get_Q(0), ctx.get_f(0), ctx.force(0))
        ctx.close()
    for tile in (5, 8):
        dq = np.max(np.abs(res[tile][0] - res[6][0]))
        df = np.max(np.abs(res[tile][1] - res[6][1]))
        say("   tile %d: max |dQ| %.3e |df| %.3e" % (tile, dq, df))
        assert dq < 1e-6 and df < 1e-7
        assert np.linalg.norm(res[tile][2] - res[6][2]) <= 1e-4 * np.linalg.norm(res[6][2]) + 1e-8


@pytest.mark.parametrize("anchoring,motion", [("normal", "fixed"), ("planar", "free")])
def test_same_bits_for_any_work_split(anchoring, motion):
    """A 128^3 box with an a = 16 colloid marched alone and next to a 64^3
    box: the second box takes resident blocks, so the first box's column
    blocks are cut into different runs of planes (work items start at other
    planes next to the colloid).  Every plane's arithmetic is the same
    wherever an item starts, so the bits agree."""
    from paper_1102_2193_amd import lc
    say("case: 128^3 fp32 a = 16 %s %s, alone vs beside a 64^3 box (different work items)" % (anchoring, motion))
    kw = dict(anchoring=anchoring, W=math.inf)
    if motion == "free":
        kw.update(motion=lc.FREE, fext=(0.0, 0.0, 0.05), rho_c=1.0)
    box = dict(nx=128, precision="fp32", **NEM)
    other = dict(nx=64, precision="fp32", **NEM)
    Q0 = inputs.uniaxial_q(128, 128, 128, inputs.Q_INIT, director=(0.0, 0.0, 1.0))
    res = []
    for boxes in ([box], [box, other]):
        ctx = lc.Context(boxes)
        ctx.set_tile(5)
        ctx.set_colloid(0, (64.0, 64.0, 64.0), 16.0, **kw)
        ctx.set_Q(0, Q0)
        if len(boxes) > 1:
            ctx.set_Q(1, inputs.noisy_nematic_q(64, 64, 64, inputs.Q_INIT, seed=9))
        ctx.step(8)
        c = ctx.get_colloid(0)
        res.append((ctx.get_Q(0), ctx.get_f(0), ctx.get_u(0), ctx.force(0), np.array(c.pos), np.array(c.vel)))
        ctx.close()
    for k, name in enumerate(("Q", "f", "u", "force", "position", "velocity")):
        np.testing.assert_array_equal(res[0][k], res[1][k], err_msg=name)


def test_batch_equals_single_boxes_and_oracle():
    from oracle import lco
    from paper_1102_2193_amd import lc
    say("case: batch of 3 uneven fp32 boxes")
    boxes = [dict(nx=24, precision="fp32", **dict(NEM, q0=2 * math.pi / 24)),
             dict(nx=16, ny=20, nz=12, precision="fp32", **NEM),
             dict(nx=32, precision="fp32", **dict(NEM, q0=2 * math.pi / 16))]
    cols = [((12, 12, 12), 4.0, "normal"), ((8, 10, 6), 3.0, "planar"), ((16, 16, 16), 6.0, "normal")]
    Qs = [inputs.helix_q(24, 24, 24, 2 * math.pi / 24, inputs.Q_INIT),
          inputs.noisy_nematic_q(16, 20, 12, inputs.Q_INIT, seed=3),
          inputs.helix_q(32, 32, 32, 2 * math.pi / 16, inputs.Q_INIT)]
    ctx = lc.Context(boxes)
    for b, (pos, a, an) in enumerate(cols):
        ctx.set_colloid(b, pos, a, anchoring=an, W=math.inf)
        ctx.set_Q(b, Qs[b])
    ctx.step(40)
    for b, (pos, a, an) in enumerate(cols):
        single = lc.Context([boxes[b]])
        single.set_colloid(0, pos, a, anchoring=an, W=math.inf)
        single.set_Q(0, Qs[b])
        single.step(40)
        np.testing.assert_array_equal(ctx.get_Q(b), single.get_Q(0))
        np.testing.assert_array_equal(ctx.get_f(b), single.get_f(0))
        single.close()
        p = {k: v for k, v in boxes[b].items() if k not in ("nx", "ny", "nz", "precision")}
        ref = lco.Sim(boxes[b]["nx"], boxes[b].get("ny"), boxes[b].get("nz"), **p)
        ref.set_colloid(pos, a, anchoring=ANCH[an], W=math.inf)
        ref.set_Q(Qs[b])
        ref.step(40)
        m = ~ref.solid()
        eq = rel_inf(ctx.get_Q(b), ref.get_Q(), m)
        ef = rel_inf(ctx.get_f(b), ref.get_f(), m)
        say("   box %d rel err Q %.3e f %.3e" % (b, eq, ef))
        assert eq < 1e-5 and ef < 1e-5


def test_graph_replay_equals_eager():
    from paper_1102_2193_amd import lc
    say("case: graph vs eager, 24^3 fp32, 37 steps")
    L = 24
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=9)
    out = []
    for g in (False, True):
        ctx = lc.Context([dict(nx=L, precision="fp32", **NEM)])
        ctx.use_graph(g)
        ctx.set_colloid(0, (12.0, 12.0, 12.0), 4.0, anchoring="normal", W=0.01, vel=(1e-2, 0, 0),
                        motion=lc.PRESCRIBED)
        ctx.set_Q(0, Q0)
        for n in (1, 36):
            ctx.step(n)
        out.append((ctx.get_Q(0), ctx.get_f(0), ctx.force_history(0, 37), np.array(ctx.get_colloid(0).pos)))
        ctx.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)


def test_graph_replays_with_eager_work_between():
    """Four replays of the 16-step graph, each followed on the same stream by
    host reads and the eager diagnostics kernels (anchoring pass and sums);
    after every replay the state, the force, the force history and the
    diagnostics equal, bit for bit, those of eager stepping with the same
    work between.  (The getters finish the last step of a run; a run ending
    on a graph replay after an earlier read once left it unfinished, so the
    force was a step old and the history a step short.)"""
    from paper_1102_2193_amd import lc
    say("case: graph replays with eager work between, 24^3 fp32, 4 x 16 steps")
    L = 24
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=19)
    runs = []
    for g in (False, True):
        ctx = lc.Context([dict(nx=L, precision="fp32", **NEM)])
        ctx.use_graph(g)
        ctx.set_colloid(0, (11.6, 12.3, 12.1), 4.0, anchoring="planar", W=0.02, vel=(1.5e-2, -5e-3, 0),
                        motion=lc.PRESCRIBED)
        ctx.set_Q(0, Q0)
        snaps = []
        for r in range(4):
            ctx.step(16)
            d = ctx.diag(0)
            snaps.append([ctx.get_Q(0), ctx.get_f(0), ctx.get_u(0), ctx.force(0), ctx.force_history(0, 16 * (r + 1)),
                          np.array([d["free_energy"], d["mass"], d["umax"], *d["momentum"]]),
                          np.array(ctx.get_colloid(0).pos)])
        runs.append(snaps)
        ctx.close()
    for r, (a, b) in enumerate(zip(*runs)):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
        say("   replay %d equal to eager" % (r + 1))


def test_graph_rebuilt_after_the_host_changes_the_setup():
    """Graph replays, then the host moves the colloid to another place (a new
    work layout), changes the tile shape and writes a new Q; the replays that
    follow equal eager stepping through the same changes, bit for bit."""
    from paper_1102_2193_amd import lc
    say("case: graph replays around set_colloid / set_tile / set_Q, 32^3 fp32")
    L = 32
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=23)
    Q1 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=24, director=(1, 0, 0))
    runs = []
    for g in (False, True):
        ctx = lc.Context([dict(nx=L, precision="fp32", **NEM)])
        ctx.use_graph(g)
        march = [t for t in range(ctx.num_tiles()) if tuple(ctx.tile_shape(t)) == (64, 8, 8)][0]
        ctx.set_colloid(0, (10.4, 12.2, 15.9), 4.0, anchoring="normal", W=0.01, vel=(0.01, 0, 0),
                        motion=lc.PRESCRIBED)
        ctx.set_Q(0, Q0)
        ctx.step(32)
        ctx.set_colloid(0, (22.3, 20.6, 8.1), 5.0, anchoring="planar", W=0.02, vel=(0, 0.01, -0.01),
                        motion=lc.PRESCRIBED)
        ctx.step(16)
        ctx.set_tile(march)
        ctx.step(16)
        ctx.set_Q(0, Q1)
        ctx.step(32)
        runs.append([ctx.get_Q(0), ctx.get_f(0), ctx.get_u(0), ctx.force(0), ctx.force_history(0, 48),
                     np.array(ctx.get_colloid(0).pos)])
        ctx.close()
    for x, y in zip(*runs):
        np.testing.assert_array_equal(x, y)


def test_diag_and_defects_match_oracle():
    say("case: diag/defects 24^3 fp64 cholesteric")
    L = 24
    prm = dict(NEM, q0=2 * math.pi / 24)
    col = dict(pos=(12.0, 12.0, 12.0), a0=5.0, anchoring="normal", W=math.inf)
    Q0 = inputs.helix_q(L, L, L, 2 * math.pi / 24, inputs.Q_INIT)
    r = run_pair((L, L, L), prm, 30, "fp64", colloid=col, Q0=Q0)
    d, dr = r["ctx"].diag(0), r["ref"].diag()
    for k in ("free_energy", "mass"):
        assert d[k] == pytest.approx(dr[k], rel=1e-11), k
    np.testing.assert_allclose(d["momentum"], dr["momentum"], atol=1e-10)
    assert d["umax"] == pytest.approx(dr["umax"], rel=1e-9)
    Q = r["ctx"].get_Q(0)
    xx, xy, xz, yy, yz = Q
    T = np.stack([np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1), np.stack([xz, yz, -xx - yy], -1)], -2)
    lam = np.linalg.eigvalsh(T)[..., 2]
    for thr in (0.435, 0.49):
        mask, cnt = r["ctx"].defects(0, thr)
        ref = (1.5 * lam < thr) & r["fluid"]
        np.testing.assert_array_equal(mask, ref)
        assert cnt == int(ref.sum())
    assert cnt > 0


def test_weak_anchoring_fp32_cholesteric64():
    say("case: 48^3 fp32 cholesteric, fixed homeotropic a=8, 60 steps")
    L = 48
    q0 = 2 * math.pi / 24
    prm = dict(NEM, q0=q0)
    col = dict(pos=(24.0, 24.0, 24.0), a0=8.0, anchoring="normal", W=math.inf)
    Q0 = inputs.helix_q(L, L, L, q0, inputs.Q_INIT)
    r = run_pair((L, L, L), prm, 60, "fp32", colloid=col, Q0=Q0, hist=True)
    check(r, 1e-5, 1e-5, tol_force=1e-3)


def test_numeric_error_is_reported():
    from paper_1102_2193_amd import lc
    say("case: NaN injection")
    L = 16
    ctx = lc.Context([dict(nx=L, precision="fp32", **NEM)])
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=1)
    Q0[0, 3, 4, 5] = np.nan
    ctx.set_Q(0, Q0)
    ctx.step(2)
    with pytest.raises(lc.LCError) as e:
        ctx.get_Q(0)
    assert e.value.code == 4


# ---------------------------------------------------------------------------
# free colloid (velocity and position from the force)
# ---------------------------------------------------------------------------
FREE = dict(motion=2, vel=(0.03, -0.02, 0.01), omega=(0.0, 0.0, 0.002), fext=(2e-3, 0.0, -1e-3), rho_c=1.3)


def _state(ctx, ref):
    c, oc = ctx.get_colloid(0), ref.get_colloid()
    return (np.array(list(c.pos) + list(c.vel) + list(c.omega)),
            np.array(list(oc.pos) + list(oc.vel) + list(oc.omega)))


def test_free_colloid_fp64_against_oracle():
    say("case: 16^3 fp64 chiral planar W=0.02, free colloid a=3.5 with external force, 40 steps")
    L = 16
    prm = dict(NEM, q0=0.2)
    col = dict(pos=(7.6, 8.3, 8.1), a0=3.5, anchoring="planar", W=0.02, S0=0.5, **FREE)
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=31, noise=0.02, director=(1, 0.2, 0.4))
    r = run_pair((L, L, L), prm, 40, "fp64", colloid=col, Q0=Q0, hist=True)
    check(r, 1e-10, 1e-12, tol_u=1e-8, tol_force=1e-8)
    g, o = _state(r["ctx"], r["ref"])
    say("   pos/vel/omega max diff %.3e" % np.max(np.abs(g - o)))
    np.testing.assert_allclose(g, o, rtol=1e-9, atol=1e-13)
    assert np.linalg.norm(g[3:6] - np.array(FREE["vel"])) > 1e-4   # it did move under the force


def test_free_colloid_fp32_marching_against_oracle():
    say("case: 32^3 fp32 normal W=0.01, free colloid a=4 pulled along x, 60 steps")
    L = 32
    col = dict(pos=(15.6, 16.3, 16.2), a0=4.0, anchoring="normal", W=0.01, S0=0.5, motion=2,
               vel=(0.0, 0.0, 0.0), fext=(0.02, 0.0, 0.0), rho_c=1.0)
    Q0 = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=32)
    r = run_pair((L, L, L), NEM, 60, "fp32", colloid=col, Q0=Q0, hist=True)
    check(r, 1e-5, 1e-5, tol_force=1e-3)
    g, o = _state(r["ctx"], r["ref"])
    say("   vel gpu %s oracle %s" % (g[3:6], o[3:6]))
    np.testing.assert_allclose(g[3:6], o[3:6], rtol=1e-4, atol=1e-9)
    np.testing.assert_allclose(g[0:3], o[0:3], atol=1e-6)
    assert o[3] > 1e-4                                             # pulled along +x


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_free_colloid_closed_form_without_fluid(precision):
    from paper_1102_2193_amd import lc
    say("case: 16^3 %s fluid off, Q = 0, free colloid with external force, 40 steps" % precision)
    L, a, rho_c, n = 16, 3.0, 1.5, 40
    fext, v0 = np.array([2e-3, -1e-3, 5e-4]), np.array([1e-3, 0.0, -2e-3])
    ctx = lc.Context([dict(nx=L, precision=precision, **dict(NEM, hydro=0))])
    ctx.set_colloid(0, (8.2, 7.9, 8.4), a, anchoring="none", motion=lc.FREE, vel=tuple(v0), fext=tuple(fext),
                    rho_c=rho_c)
    ctx.set_Q(0, np.zeros((5, L, L, L)))
    ctx.step(n)
    c = ctx.get_colloid(0)
    acc = fext / (4.0 / 3.0 * math.pi * a ** 3 * rho_c)
    np.testing.assert_allclose(np.array(c.vel), v0 + n * acc, rtol=1e-12, atol=1e-17)
    np.testing.assert_allclose(np.array(c.pos), (np.array([8.2, 7.9, 8.4]) + n * v0 + acc * n * (n + 1) / 2) % L,
                               atol=1e-12)
    assert np.all(ctx.force_history(0, n) == 0.0)
    ctx.close()


def test_free_colloid_conserves_total_momentum():
    from paper_1102_2193_amd import lc
    say("case: 16^3 fp64 free colloid, no external force: fluid + colloid momentum, 20 steps")
    L, a = 16, 3.5
    ctx = lc.Context([dict(nx=L, precision="fp64", **NEM)])
    ctx.set_colloid(0, (8.3, 7.6, 8.1), a, anchoring="planar", W=0.01, motion=lc.FREE, vel=(0.06, 0.0, -0.03))
    ctx.set_Q(0, inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, 21, noise=0.02))
    M = 4.0 / 3.0 * math.pi * a ** 3 * NEM.get("rho0", 1.0)

    def total():
        return ctx.diag(0)["momentum"] + M * np.array(ctx.get_colloid(0).vel)
    p0 = total()
    for _ in range(20):
        ctx.step(1)
        np.testing.assert_allclose(total(), p0, atol=1e-11)
    ctx.close()
