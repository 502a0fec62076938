"""Pins of the oracle with several colloids in one box.

The paper's outlook (Introduction; Sec. 3.2, closing paragraph) is colloid-
colloid interactions through the liquid crystal.  The oracle holds up to 16
colloids per box whose surfaces stay at least 3 lattice units apart, so that
every link, face and ghost node belongs to one colloid.  Fixed here by:

* brute force: the solid map tags each node with its colloid;
* locality: two colloids farther apart than the stencils reach, in a
  uniform field with the fluid at rest, each get exactly the force and
  torque of the same colloid alone in the box (first step);
* translation: a copy of a colloid shifted by a lattice vector gets the same
  force;
* momentum: per step the fluid momentum changes by minus the sum of all
  colloid forces (fixed and prescribed motion with events), and fluid plus
  colloid momentum is conserved for free colloids;
* the separation rule: too-close colloids are refused at set-up, and a step
  that would start with them too close is refused.
"""
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs
from test_oracle_pins_transport import solid_map

NEM = inputs.NEMATIC


def test_solid_map_tags_each_colloid(oracle):
    L = 24
    specs = [dict(pos=(6.3, 7.1, 5.8), a0=3.2), dict(pos=(16.6, 15.2, 17.4), a0=4.4),
             dict(pos=(5.5, 18.3, 16.9), a0=2.7)]
    s = oracle.Sim(L, **NEM)
    s.set_colloids(specs)
    want = np.zeros((L, L, L), dtype=np.uint8)
    for k, sp in enumerate(specs):
        want[solid_map((L, L, L), sp["pos"], sp["a0"])] = k + 1
    np.testing.assert_array_equal(s.solid_id(), want)
    assert s.num_colloids() == 3 and [c.a0 for c in s.get_colloids()] == [3.2, 4.4, 2.7]


@pytest.mark.parametrize("anch,motion", [("normal", 0), ("planar", 0), ("planar", 1)])
def test_distant_colloids_each_feel_their_own_force(oracle, anch, motion):
    L = 32
    an = {"normal": oracle.ANCHOR_NORMAL, "planar": oracle.ANCHOR_PLANAR}[anch]
    A = dict(pos=(8.3, 8.6, 9.1), a0=4.2, anchoring=an, W=0.02, S0=0.5)
    B = dict(pos=(22.4, 23.7, 21.2), a0=5.1, anchoring=oracle.ANCHOR_NORMAL, W=math.inf, S0=0.5)
    if motion:   # different rigid-body motions, with moving-boundary events in the step
        A.update(motion=oracle.PRESCRIBED, vel=(0.4, -0.1, 0.2), omega=(0.0, 0.01, -0.02))
        B.update(motion=oracle.PRESCRIBED, vel=(-0.2, 0.3, 0.35), omega=(0.015, 0.0, 0.01))
    Q = inputs.uniaxial_q(L, L, L, inputs.Q_INIT, director=(0.2, 0.3, 1.0))
    both = oracle.Sim(L, **NEM)
    both.set_colloids([A, B])
    both.set_Q(Q)
    both.step(1)
    F = both.forces()
    for k, sp in enumerate((A, B)):
        alone = oracle.Sim(L, **NEM)
        alone.set_colloids([sp])
        alone.set_Q(Q)
        alone.step(1)
        np.testing.assert_array_equal(F[k], alone.forces()[0])
        assert np.linalg.norm(F[k]) > 1e-6


def test_lattice_translated_copy_feels_the_same_force(oracle):
    L = 32
    A = dict(pos=(8.3, 8.6, 9.1), a0=4.6, anchoring=oracle.ANCHOR_PLANAR, W=0.03, S0=0.5)
    B = dict(A, pos=(8.3 + 16, 8.6 + 16, 9.1))
    Q = inputs.uniaxial_q(L, L, L, inputs.Q_INIT, director=(0.3, 0.1, 1.0))
    s = oracle.Sim(L, **NEM)
    s.set_colloids([A, B])
    s.set_Q(Q)
    for _ in range(3):
        s.step(1)
        F = s.forces()
        np.testing.assert_allclose(F[1], F[0], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("motion", [0, 1])
def test_fluid_momentum_balances_all_colloid_forces(oracle, motion):
    L = 24
    prm = dict(NEM, q0=0.15)
    specs = [dict(pos=(6.3, 7.1, 5.8), a0=3.2, anchoring=oracle.ANCHOR_PLANAR, W=0.02, S0=0.5,
                  vel=(0.09, 0.0, -0.05) if motion else (0, 0, 0), omega=(0, 0.004, 0), motion=motion),
             dict(pos=(16.6, 15.2, 17.4), a0=4.4, anchoring=oracle.ANCHOR_NORMAL, W=math.inf, S0=0.5,
                  vel=(-0.04, 0.07, 0.0) if motion else (0, 0, 0), omega=(0.003, 0, 0), motion=motion),
             dict(pos=(5.5, 18.3, 16.9), a0=2.7, anchoring=oracle.ANCHOR_NORMAL, W=0.05, S0=0.5)]
    s = oracle.Sim(L, **prm)
    s.set_colloids(specs)
    s.set_Q(inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=91, noise=0.02))
    c, _ = oracle.lattice()
    d0 = s.diag()
    for _ in range(8):
        p0 = d0["momentum"]
        s.step(1)
        d0 = s.diag()
        dp = d0["momentum"] - p0
        F = s.forces()
        np.testing.assert_allclose(dp, -(F[:, 0:3] + F[:, 3:6]).sum(axis=0), rtol=0, atol=1e-12)
    if motion:
        pos = np.array([list(k.pos) for k in s.get_colloids()])
        start = np.array([sp["pos"] for sp in specs])
        assert np.all(np.abs(pos - start)[:2].max(axis=1) > 0.3)


def test_free_colloids_conserve_total_momentum(oracle):
    L = 24
    specs = [dict(pos=(6.3, 7.1, 5.8), a0=3.2, anchoring=oracle.ANCHOR_PLANAR, W=0.02, motion=oracle.FREE,
                  vel=(0.05, 0.0, -0.02), rho_c=1.2),
             dict(pos=(16.6, 15.2, 17.4), a0=4.4, anchoring=oracle.ANCHOR_NORMAL, W=0.01, motion=oracle.FREE,
                  vel=(-0.03, 0.04, 0.0), rho_c=0.9)]
    s = oracle.Sim(L, **NEM)
    s.set_colloids(specs)
    s.set_Q(inputs.noisy_nematic_q(L, L, L, inputs.Q_INIT, seed=92, noise=0.02))
    M = [4.0 / 3.0 * math.pi * sp["a0"] ** 3 * sp["rho_c"] for sp in specs]

    def total():
        return s.diag()["momentum"] + sum(m * np.array(c.vel) for m, c in zip(M, s.get_colloids()))
    p0 = total()
    for _ in range(15):
        s.step(1)
        np.testing.assert_allclose(total(), p0, rtol=0, atol=1e-11)


def test_separation_rule_refuses(oracle):
    L = 24
    s = oracle.Sim(L, **NEM)
    with pytest.raises(ValueError):
        s.set_colloids([dict(pos=(8.0, 8.0, 8.0), a0=3.0), dict(pos=(16.5, 8.0, 8.0), a0=3.0)])   # gap 2.5
    s.set_colloids([dict(pos=(8.0, 8.0, 8.0), a0=3.0), dict(pos=(17.2, 8.0, 8.0), a0=3.0)])       # gap 3.2
    # moving towards each other: the first step that starts closer than 3 is refused
    s.set_colloids([dict(pos=(8.0, 8.0, 8.0), a0=3.0, vel=(0.25, 0, 0), motion=oracle.PRESCRIBED),
                    dict(pos=(17.2, 8.0, 8.0), a0=3.0)])
    s.step(1)                     # starts at a gap of 3.2, ends at 2.95
    with pytest.raises(RuntimeError):
        s.step(5)
    assert s.nstep == 1
