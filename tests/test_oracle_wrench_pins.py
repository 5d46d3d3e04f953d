"""Pins of the oracle's twist and joint-wrench maps (rigid-motion embedding
E(A) of Eq. module2-E, twist map G(A) of Eq. module1-G-twist, virtual work as
in the single-body comparison of Sec. 6).

  * a rigid body spinning at omega with velocity v has the twist [omega; v]
    (closed form, any orientation);
  * a ball joint's force on a body is the point force -/+ lambda at the
    anchor: its wrench about the centre of mass is [r x F; F] with r the
    anchor's world offset A p (plain statics, computed here in numpy);
  * internal joints act in equal and opposite pairs: on a free assembly the
    joint forces of all bodies sum to zero (ball and hinge), and with ball
    joints at coincident anchors their moments about the origin too;
  * a box hanging at rest from a world ball joint above its centre carries its
    weight: the joint wrench is the weight's opposite, with no torque.
"""
import numpy as np

import mabd_inputs as mi
import oracle
from test_oracle_pins import rot


def test_twist_of_rigid_spin():
    rng = np.random.default_rng(3)
    for _ in range(5):
        R = rot(rng.normal(size=3), rng.uniform(0, np.pi))
        om, v = rng.normal(size=3), rng.normal(size=3)
        b = mi.free_body(dims=(0.3, 0.2, 0.1), A=R)
        qd = np.zeros((1, 12))
        for c in range(3):
            qd[0, 3 * c:3 * c + 3] = np.cross(om, R[:, c])
        qd[0, 9:] = v
        V = oracle.System(b).twists(b.q0, qd)
        assert np.allclose(V[0, :3], om, rtol=0, atol=1e-14)
        assert np.allclose(V[0, 3:], v, rtol=0, atol=1e-15)


def test_ball_joint_wrench_is_the_anchor_point_force():
    """Two bodies, one ball joint, tilted poses: the wrench on side a is the
    moment of -lambda applied at A_a p_a, on side b that of +lambda at A_b p_b."""
    asm = mi.chain(3, seed=5, pin_first=False)
    rng = np.random.default_rng(6)
    q = asm.q0.copy()
    for b in range(asm.n):
        q[b, :9] = rot(rng.normal(size=3), 0.4).T.reshape(9)
    s = oracle.System(asm)
    lam = rng.normal(size=s.rows)
    W = s.joint_wrenches(q, lam)
    expect = np.zeros((asm.n, 6))
    for k in range(asm.m):
        L = lam[3 * k:3 * k + 3]
        for b, p, sgn in ((asm.ja[k], asm.pa[k], -1.0), (asm.jb[k], asm.pb[k], 1.0)):
            A = q[b, :9].reshape(3, 3).T
            F = sgn * L
            expect[b, :3] += np.cross(A @ p, F)
            expect[b, 3:] += F
    assert np.allclose(W, expect, rtol=0, atol=1e-13 * np.abs(expect).max())


def test_internal_joint_forces_cancel():
    rng = np.random.default_rng(7)
    # mixed ball / hinge chain without pinned bodies: forces sum to zero
    asm = mi.chain(12, seed=8, hinge_frac=0.5, pin_first=False)
    s = oracle.System(asm)
    q, qd, _, _ = s.step(asm.h, asm.q0, asm.q0 * 0 + rng.normal(0, 0.05, asm.q0.shape))
    lam = rng.normal(size=s.rows)
    W = s.joint_wrenches(q, lam)
    assert np.abs(W[:, 3:].sum(axis=0)).max() <= 1e-13 * np.abs(W[:, 3:]).max()
    # all-ball chain at a state where the anchors coincide (after a step):
    # the moments about the origin cancel as well
    ab = mi.chain(12, seed=9, pin_first=False)
    sb = oracle.System(ab)
    qb, _, _, _ = sb.step(ab.h, ab.q0, ab.qd0 + rng.normal(0, 0.05, ab.qd0.shape))
    lb = rng.normal(size=sb.rows)
    Wb = sb.joint_wrenches(qb, lb)
    mom = (np.cross(qb[:, 9:], Wb[:, 3:]) + Wb[:, :3]).sum(axis=0)
    assert np.abs(Wb[:, 3:].sum(axis=0)).max() <= 1e-13 * np.abs(Wb[:, 3:]).max()
    assert np.abs(mom).max() <= 1e-11 * np.abs(Wb).max()


def test_hanging_box_carries_its_weight():
    """A stiff 1 m box hanging at rest from a world ball joint at its top face
    (a softer box would first stretch under its weight, and the joint would
    carry the weight less the stretch mode's inertia)."""
    b = mi.free_body(dims=(0.1, 0.1, 1.0), k_orth=1e14)  # near rigid: at rest, in equilibrium
    b.jtype = np.array([0], np.uint8)
    b.ja = np.array([0], np.int32); b.jb = np.array([-1], np.int32)
    b.pa = np.array([[0.0, 0.0, 0.5]]); b.pb = np.array([[0.0, 0.0, 0.5]])
    b.axis = np.array([[0.0, 1.0, 0.0]]); b.cp_len = np.array([0.1])
    s = oracle.System(b)
    q1, qd1, lam, d = s.step(b.h, b.q0, b.qd0)
    W = s.joint_wrenches(b.q0, lam)
    weight = 1000.0 * 0.01 * 9.8
    assert abs(W[0, 5] - weight) <= 1e-6 * weight, W
    assert np.abs(W[0, 3:5]).max() <= 1e-9 * weight
    assert np.abs(W[0, :3]).max() <= 1e-9 * weight
