"""Pins of the oracle's higher-order variants of two readings of Sec. 2.2.

* Advection (the advective fluxes at control-volume faces): second-order
  upwind and third-order upwind-biased face values.  For a uniform velocity
  one step is the textbook difference of that order (closed form, per axis
  and sign), its error on a smooth wave falls as the order says, and next to
  a colloid the fluid sum of Q is still conserved (no flux through solid
  faces, fluxes shared by the two nodes of a face).
* The Q stencil ("the same stencil" used everywhere in the fluid): the
  isotropic 27-point gradient and Laplacian are exact on quadratics, their
  Laplacian is direction-independent to a far higher degree than the compact
  7-point one on two waves of equal |k|, and ghost Q reaches every solid node
  that a fluid node's 27-point stencil touches.
"""
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs
from test_oracle_pins_transport import INERT, solid_map

NEM = inputs.NEMATIC


def upwind_step(Q, U, order):
    """One explicit step of the upwind difference of the given order for a
    uniform velocity U (textbook forms, per axis)."""
    out = Q.copy()
    for b, axis in ((0, 3), (1, 2), (2, 1)):
        if U[b] == 0.0:
            continue
        s = 1 if U[b] > 0 else -1
        back = np.roll(Q, s, axis=axis)        # Q(x - s e)
        back2 = np.roll(Q, 2 * s, axis=axis)   # Q(x - 2 s e)
        fwd = np.roll(Q, -s, axis=axis)        # Q(x + s e)
        if order == 2:
            d = (3 * Q - 4 * back + back2) / 2
        else:
            d = (2 * fwd + 3 * Q - 6 * back + back2) / 6
        out -= abs(U[b]) * d
    return out


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("U", [(0.03, 0.0, 0.0), (-0.05, 0.0, 0.0), (0.0, 0.04, 0.0), (0.0, 0.0, -0.02),
                               (0.031, -0.017, 0.045)])
def test_higher_order_upwind_closed_form(oracle, order, U):
    nx, ny, nz = 7, 8, 9
    s = oracle.Sim(nx, ny, nz, advection=order, **INERT)
    Q = inputs.noisy_nematic_q(nx, ny, nz, 0.3, seed=71, noise=0.2, director=(2, 1, 3))
    s.set_Q(Q)
    u = np.empty((3, nz, ny, nx))
    for a in range(3):
        u[a] = U[a]
    s.set_u(u)
    s.step(1)
    np.testing.assert_allclose(s.get_Q(), upwind_step(Q, U, order), rtol=0, atol=4e-16)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_upwind_error_falls_with_the_order(oracle, order):
    """A wave Q = A sin(k x) advected one step by a small uniform U along x:
    (Q - Q_new)/U estimates dQ/dx; doubling the wavelength (in sites)
    divides the relative error by 2^order."""
    errs = []
    for L in (32, 64):
        s = oracle.Sim(L, 4, 4, advection=order, **INERT)
        k = 2 * math.pi / L
        x = np.arange(L)
        Q = np.zeros((5, 4, 4, L))
        Q[1] = 0.1 * np.sin(k * x)[None, None, :]
        s.set_Q(Q)
        U = 1e-3
        u = np.zeros((3, 4, 4, L))
        u[0] = U
        s.set_u(u)
        s.step(1)
        est = (Q[1] - s.get_Q()[1]) / U
        exact = 0.1 * k * np.cos(k * x)[None, None, :]
        errs.append(np.max(np.abs(est - exact)) / (0.1 * k))
    ratio = errs[0] / errs[1]
    assert ratio == pytest.approx(2.0 ** order, rel=0.1), (order, errs, ratio)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_higher_order_fluxes_conserve_the_fluid_sum_next_to_a_colloid(oracle, order):
    L, a = 14, 3.6
    U = (0.011, -0.007, 0.004)
    R = (6.95, 7.15, 6.85)
    s = oracle.Sim(L, advection=order, **INERT)
    s.set_colloid(R, a, anchoring=oracle.ANCHOR_NONE, vel=U, motion=oracle.PRESCRIBED)
    Q = inputs.noisy_nematic_q(L, L, L, 0.4, seed=43, noise=0.15, director=(0.3, 1.0, 0.2))
    s.set_Q(Q)
    u = np.empty((3, L, L, L))
    for k in range(3):
        u[k] = U[k]
    s.set_u(u)
    before = s.solid()
    s.step(1)
    np.testing.assert_array_equal(before, s.solid())
    fluid = ~before
    np.testing.assert_allclose(s.get_Q()[:, fluid].sum(axis=1), Q[:, fluid].sum(axis=1), rtol=0, atol=5e-12)
    if order > 1:
        # away from the colloid the step is the closed form of its order
        far = ~solid_map(before.shape, R, a + 4.0)
        ref = upwind_step(Q, U, order)
        np.testing.assert_allclose(s.get_Q()[:, far], ref[:, far], rtol=0, atol=4e-16)


@pytest.mark.parametrize("order", [2, 3])
def test_wide_stencils_reaching_the_colloid_fall_back_to_first_order(oracle, order):
    """Uniform Q in the fluid, other values at the solid nodes (fixed
    homeotropic ghosts), one uniform velocity for fluid and colloid: every
    face between two fluid nodes must carry U Q_fluid, also where the wider
    upwind stencil would reach into the colloid, so only fluid nodes with a
    solid face neighbour (zero flux there) change."""
    L, a = 14, 3.6
    U = (0.011, -0.007, 0.004)
    R = (6.95, 7.15, 6.85)
    s = oracle.Sim(L, advection=order, **INERT)
    s.set_colloid(R, a, anchoring=oracle.ANCHOR_NORMAL, W=math.inf, S0=0.5, vel=U, motion=oracle.PRESCRIBED)
    Q = inputs.uniaxial_q(L, L, L, 0.4, director=(0.3, 1.0, 0.2))
    s.set_Q(Q)
    u = np.empty((3, L, L, L))
    for k in range(3):
        u[k] = U[k]
    s.set_u(u)
    solid = s.solid()
    s.step(1)
    touching = np.zeros_like(solid)
    for axis in range(3):
        for sh in (1, -1):
            touching |= np.roll(solid, sh, axis=axis)
    inner = ~solid & ~touching
    reach2 = np.zeros_like(solid)
    for axis in range(3):
        for sh in (2, -2):
            reach2 |= np.roll(solid, sh, axis=axis)
    assert (inner & reach2).sum() > 20          # wide stencils that reach a solid node
    np.testing.assert_array_equal(s.get_Q()[:, inner], Q[:, inner])


def _laplacian_at(oracle, Q, stencil, site):
    """K lap Q at one site from the oracle's molecular field (A0 = q0 = 0,
    K = 1: H is the Laplacian)."""
    nz, ny, nx = Q.shape[1:]
    s = oracle.Sim(nx, ny, nz, hydro=0, stencil=stencil, **dict(NEM, A0=0.0, K=1.0, q0=0.0))
    s.set_Q(Q)
    H, _, _ = s.fields()
    z, y, x = site
    return H[:, z, y, x]


def test_27_point_operators_exact_on_quadratics(oracle):
    L = 12
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    X, Y, Z = x - 6.0, y - 5.0, z - 6.0
    Q = np.zeros((5, L, L, L))
    Q[0] = 0.01 * (X * X + 2 * Y * Z - 0.5 * Z * Z + X)        # lap = 0.01 (2 - 1) = 0.01
    Q[1] = 0.02 * (X * Y + Y * Y)                               # lap = 0.04
    Q[2] = 0.005 * (Z * Z + X * Z - Y)                          # lap = 0.01
    Q[3] = -0.01 * (Y * Y + X * X + Z * Z)                      # lap = -0.06
    Q[4] = 0.03 * (X * Z + Y)                                   # lap = 0
    lap = _laplacian_at(oracle, Q, 27, (6, 5, 6))
    np.testing.assert_allclose(lap, [0.01, 0.04, 0.01, -0.06, 0.0], rtol=0, atol=1e-15)
    # the gradient enters the stress: P_zz of a pure gradient field is
    # -K |d_z Q|^2 + K/2 |dQ|^2 (A0 = xi = q0 = 0), exact with exact gradients
    s = oracle.Sim(L, hydro=1, stencil=27, **dict(NEM, A0=0.0, K=1.0, q0=0.0, xi=0.0))
    s.set_Q(Q)
    _, P, _ = s.fields()
    # analytic first derivatives at the site (X, Y, Z) = (0, 0, 0)
    dx = np.array([0.01, 0.0, 0.0, 0.0, 0.0])
    dy = np.array([0.0, 0.0, -0.005, 0.0, 0.03])
    dz = np.array([0.0, 0.0, 0.0, 0.0, 0.0])

    def full2(v):
        return v[0] ** 2 + v[3] ** 2 + (v[0] + v[3]) ** 2 + 2 * (v[1] ** 2 + v[2] ** 2 + v[4] ** 2)
    tot = full2(dx) + full2(dy) + full2(dz)
    Pzz = -full2(dz) + 0.5 * tot
    Pxx = -full2(dx) + 0.5 * tot
    assert P[8, 6, 5, 6] == pytest.approx(Pzz, abs=1e-15)
    assert P[0, 6, 5, 6] == pytest.approx(Pxx, abs=1e-15)


def test_27_point_laplacian_is_isotropic(oracle):
    """Waves of equal |k| along (5,0,0) and (3,4,0) (box 40): the compact
    Laplacian's eigenvalues differ by 2.4%; the isotropic 27-point ones agree
    to O(k^6)."""
    L = 40
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    lam = {}
    for st in (7, 27):
        for m in ((5, 0, 0), (3, 4, 0), (0, 3, 4)):
            ph = 2 * math.pi * (m[0] * x + m[1] * y + m[2] * z) / L
            Q = np.zeros((5, L, L, L))
            Q[1] = 0.01 * np.cos(ph)
            lam[(st, m)] = _laplacian_at(oracle, Q, st, (0, 0, 0))[1] / 0.01
    k2 = (2 * math.pi * 5 / L) ** 2
    a7 = abs(lam[(7, (5, 0, 0))] - lam[(7, (3, 4, 0))]) / k2
    a27 = abs(lam[(27, (5, 0, 0))] - lam[(27, (3, 4, 0))]) / k2
    assert a7 > 0.015
    assert a27 < a7 / 20
    assert lam[(27, (3, 4, 0))] == pytest.approx(lam[(27, (0, 3, 4))], rel=1e-12)
    # the gradient: trace P = K/2 |DQ|^2 (A0 = xi = q0 = 0), so the squared
    # effective wavenumber of the difference operator is read off P
    g = {}
    for st in (7, 27):
        for m in ((5, 0, 0), (3, 4, 0)):
            ph = 2 * math.pi * (m[0] * x + m[1] * y + m[2] * z) / L
            Q = np.zeros((5, L, L, L))
            Q[1] = 0.01 * np.cos(ph)
            sim = oracle.Sim(L, hydro=1, stencil=st, **dict(NEM, A0=0.0, K=1.0, q0=0.0, xi=0.0))
            sim.set_Q(Q)
            _, P, _ = sim.fields()
            tr = P[0, 0, 0, 1] + P[4, 0, 0, 1] + P[8, 0, 0, 1]
            th = 2 * math.pi * m[0] / L
            g[(st, m)] = tr / (0.5 * 2 * 0.01 ** 2 * math.sin(th) ** 2)
    g7 = abs(g[(7, (5, 0, 0))] - g[(7, (3, 4, 0))]) / k2
    g27 = abs(g[(27, (5, 0, 0))] - g[(27, (3, 4, 0))]) / k2
    assert g7 > 0.05 and g27 < g7 / 10, (g7, g27)
    # both are second-order approximations of -k^2
    for st in (7, 27):
        assert lam[(st, (5, 0, 0))] == pytest.approx(-k2, rel=0.08)


def test_27_point_ghost_nodes_include_diagonal_contacts(oracle):
    """With the 27-point stencil every solid node with a fluid node among its
    26 neighbours holds Q^0 (fixed homeotropic anchoring); with the 7-point
    stencil, nodes whose only fluid neighbours are diagonal keep their value."""
    L, a = 16, 4.3
    R = (7.6, 8.2, 7.9)
    Q = inputs.uniaxial_q(L, L, L, 0.3, director=(0, 0, 1))
    solid = solid_map((L, L, L), R, a)
    face_contact = np.zeros_like(solid)
    any_contact = np.zeros_like(solid)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                nb_fluid = ~np.roll(solid, (-dz, -dy, -dx), axis=(0, 1, 2))
                any_contact |= nb_fluid
                if abs(dx) + abs(dy) + abs(dz) == 1:
                    face_contact |= nb_fluid
    diag_only = solid & any_contact & ~face_contact
    assert diag_only.sum() > 0
    out = {}
    for st in (7, 27):
        s = oracle.Sim(L, hydro=0, stencil=st, **NEM)
        s.set_colloid(R, a, anchoring=oracle.ANCHOR_NORMAL, W=math.inf, S0=0.5)
        s.set_Q(Q)
        out[st] = s.ghost()
    for z, y, x in zip(*np.nonzero(diag_only)):
        r = np.array([x, y, z], float) - np.array(R)
        n = r / np.linalg.norm(r)
        q0 = 0.5 * (np.outer(n, n) - np.eye(3) / 3)
        want = np.array([q0[0, 0], q0[0, 1], q0[0, 2], q0[1, 1], q0[1, 2]])
        np.testing.assert_allclose(out[27][:, z, y, x], want, rtol=0, atol=1e-15)
        np.testing.assert_array_equal(out[7][:, z, y, x], Q[:, z, y, x])
    # nodes with a fluid face neighbour get the same ghost value either way
    both = solid & face_contact
    np.testing.assert_allclose(out[27][:, both], out[7][:, both], rtol=0, atol=1e-15)
