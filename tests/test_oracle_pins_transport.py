"""Pins of the oracle's transport and moving-boundary steps (Sec. 2.2).

The advective part of the Beris-Edwards update (face fluxes, first-order
upwind, zero normal flux through solid faces) and the values given to the
nodes a moving colloid uncovers are fixed here by closed forms, a
conservation law and brute force on tiny boxes, each independent of the
oracle's own code:

* uniform velocity, no colloid, H = 0: one step is the exact upwind shift
  Q - sum_b |U_b| (Q - Q(x - sign(U_b) e_b));
* uniform velocity equal to the colloid's (no velocity gradient anywhere),
  H = 0: the sum of Q over the fluid is conserved to round-off, which holds
  only if no flux crosses a solid face;
* a prescribed move without flow, against a fixed colloid from the same
  start: an uncovered node holds the mean of its face neighbours that are
  fluid before and after the move; with flow it holds equilibrium
  populations at rho0 and the rigid-body velocity about the new centre.
"""
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs

NEM = inputs.NEMATIC
# no molecular field: A0 = K = 0 (H = 0 and the stress vanishes), Gamma = 0
INERT = dict(NEM, A0=0.0, K=0.0, Gamma=0.0)


def solid_map(shape, R, a):
    """Brute-force sphere test |x - R|^2 < a^2 with the minimum image."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = np.zeros(shape)
    for coord, c, L in ((x, R[0], nx), (y, R[1], ny), (z, R[2], nz)):
        d = coord - c
        d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
        d2 = d2 + d * d
    return d2 < a * a


@pytest.mark.parametrize("U", [(0.03, 0.0, 0.0), (-0.05, 0.0, 0.0), (0.0, 0.04, 0.0), (0.0, 0.0, -0.02),
                               (0.031, -0.017, 0.045), (-0.02, 0.06, -0.013)])
def test_upwind_advection_closed_form(oracle, U):
    """Sec. 2.2 (advective fluxes at control-volume faces), first-order
    upwind with the face velocity the mean of its two nodes: for a uniform
    velocity and H = 0 one step moves Q exactly by the upwind difference
    along each axis; a downwind or sign mistake on any axis fails."""
    nx, ny, nz = 6, 7, 8
    s = oracle.Sim(nx, ny, nz, **INERT)
    Q = inputs.noisy_nematic_q(nx, ny, nz, 0.3, seed=41, noise=0.2, director=(1, 2, 3))
    s.set_Q(Q)
    u = np.empty((3, nz, ny, nx))
    for a in range(3):
        u[a] = U[a]
    s.set_u(u)
    s.step(1)
    ref = Q.copy()
    for b, axis in ((0, 3), (1, 2), (2, 1)):
        if U[b] == 0.0:
            continue
        sg = 1 if U[b] > 0 else -1
        upwind = np.roll(Q, sg, axis=axis)   # Q(x - sg e_b)
        ref -= abs(U[b]) * (Q - upwind)
    np.testing.assert_allclose(s.get_Q(), ref, rtol=0, atol=2e-16)


def test_no_advective_flux_through_solid_faces(oracle):
    """Sec. 2.2 (zero normal flux at solid faces): fluid and colloid move
    with one uniform velocity, so the velocity gradient vanishes everywhere
    (rigid-body velocity at solid nodes) and H = 0: Q changes only by the
    face fluxes, which cancel in pairs between fluid nodes.  The sum of Q
    over the fluid is then conserved, and only then: the fluxes a solid
    face would carry are checked to be far from zero."""
    L, a = 14, 3.6
    U = (0.011, -0.007, 0.004)
    R = (6.95, 7.15, 6.85)
    s = oracle.Sim(L, **INERT)
    s.set_colloid(R, a, anchoring=oracle.ANCHOR_NONE, vel=U, motion=oracle.PRESCRIBED)
    Q = inputs.noisy_nematic_q(L, L, L, 0.4, seed=43, noise=0.15, director=(0.3, 1.0, 0.2))
    s.set_Q(Q)
    u = np.empty((3, L, L, L))
    for k in range(3):
        u[k] = U[k]
    s.set_u(u)
    before = s.solid()
    s.step(1)
    after = s.solid()
    np.testing.assert_array_equal(before, after)   # no node crosses the surface in this step
    fluid = ~before
    assert np.array_equal(before, solid_map(before.shape, R, a))
    s0 = Q[:, fluid].sum(axis=1)
    s1 = s.get_Q()[:, fluid].sum(axis=1)
    # round-off bound: ~2.5k fluid terms of size <= 1, each step's sum
    # reordered: N eps ~ 6e-13
    np.testing.assert_allclose(s1, s0, rtol=0, atol=5e-12)
    # what solid faces would carry if they were not closed: the upwind
    # fluxes ubar * Q_up summed over the fluid-solid faces (outward from the
    # fluid), with the ghost Q (mean of fluid neighbours) at solid nodes
    Qg = s.ghost()  # ghost values of the current state; only their order of size matters
    leak = np.zeros(5)
    for b, axis in ((0, 3), (1, 2), (2, 1)):
        for sg in (1, -1):
            nb_solid = np.roll(before, -sg, axis=axis - 1)     # node x + sg e_b solid
            face = fluid & nb_solid
            ub = U[b]
            out = sg * ub                                       # outward normal velocity
            q_up = np.where(out >= 0, 1.0, 0.0) * Qg + np.where(out < 0, 1.0, 0.0) * np.roll(Qg, -sg, axis=axis)
            leak += out * q_up[:, face].sum(axis=1)
    assert np.max(np.abs(leak)) > 1e-4


def _events_case(oracle, hydro, vel, omega):
    L, a = 12, 3.3
    R = (5.7, 6.2, 6.05)
    prm = dict(NEM, hydro=hydro, q0=0.1)
    Q = inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=45, noise=0.05, director=(1, 0.4, 0.7))
    runs = []
    for motion in (oracle.PRESCRIBED, oracle.FIXED):
        s = oracle.Sim(L, **prm)
        s.set_colloid(R, a, anchoring=oracle.ANCHOR_NORMAL, W=0.02, vel=vel, omega=omega, motion=motion)
        s.set_Q(Q)
        s.step(1)
        runs.append(s)
    Rn = tuple((R[k] + vel[k]) % L for k in range(3))
    old = solid_map((L, L, L), R, a)
    new = solid_map((L, L, L), Rn, a)
    return L, Rn, old, new, runs


def test_uncovered_node_q_is_mean_of_persistent_fluid_neighbours(oracle):
    """Sec. 2.2 (new fluid nodes get Q by interpolation of nearby values),
    read as the mean over the face neighbours that are fluid before and
    after the move.  Without flow the Q update does not see the colloid's
    velocity, so a fixed colloid from the same start gives the same Q^{n+1}
    at every fluid node; the moving run must agree with it away from the
    events and hold the neighbour means at uncovered nodes."""
    L, Rn, old, new, (mov, fix) = _events_case(oracle, 0, vel=(0.45, -0.3, 0.25), omega=(0, 0, 0))
    np.testing.assert_array_equal(mov.solid(), new)
    uncovered = old & ~new
    covered = new & ~old
    assert uncovered.sum() >= 10 and covered.sum() >= 10
    Qm, Qf = mov.get_Q(), fix.get_Q()
    keep = ~old & ~new
    np.testing.assert_array_equal(Qm[:, keep], Qf[:, keep])
    for z, y, x in zip(*np.nonzero(uncovered)):
        acc, n = np.zeros(5), 0
        for dz, dy, dx in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
            j = ((z + dz) % L, (y + dy) % L, (x + dx) % L)
            if old[j] or new[j]:
                continue
            acc += Qf[(slice(None),) + j]
            n += 1
        expect = acc / n if n else np.zeros(5)
        np.testing.assert_allclose(Qm[:, z, y, x], expect, rtol=1e-14, atol=1e-16)


def test_uncovered_node_fluid_moves_with_the_wall(oracle):
    """Sec. 2.2: a node the colloid uncovers becomes fluid at the reference
    density moving with the surface: equilibrium populations at rho0 and the
    rigid-body velocity v + omega x r about the new centre, and that velocity
    as its u; a node it covers holds no fluid."""
    vel, omega = (0.35, 0.2, -0.3), (0.01, -0.02, 0.015)
    L, Rn, old, new, (mov, _) = _events_case(oracle, 1, vel=vel, omega=omega)
    uncovered = old & ~new
    covered = new & ~old
    assert uncovered.sum() >= 10 and covered.sum() >= 10
    f, u = mov.get_f(), mov.get_u()
    c, w = oracle.lattice()
    for z, y, x in zip(*np.nonzero(uncovered)):
        r = np.array([x, y, z], float) - np.array(Rn)
        r = np.where(r > 0.5 * L, r - L, np.where(r < -0.5 * L, r + L, r))
        ub = np.array(vel) + np.cross(np.array(omega), r)
        np.testing.assert_allclose(u[:, z, y, x], ub, rtol=0, atol=1e-15)
        fi = f[:, z, y, x]
        np.testing.assert_allclose(fi, oracle.feq(1.0, ub), rtol=0, atol=1e-15)
        # the populations carry density rho0 and momentum rho0 u_b
        assert fi.sum() == pytest.approx(1.0, abs=1e-14)
        np.testing.assert_allclose(fi @ c, ub, rtol=0, atol=1e-14)
    assert np.all(f[:, covered] == 0.0) and np.all(u[:, covered] == 0.0)
