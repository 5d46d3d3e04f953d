"""Pins of the oracle's universal (Eq. universal) and prismatic (Eq.
prismatic) joints, next to the hinge's (Sec. 4.3) in test_oracle_pins.py.

  * kinematics, by construction of the joints (Secs. 4.4, 4.5): the motions a
    joint permits leave every row at zero, and each blocked motion moves the
    rows that block it;
  * gradients: central differences of the constraint value along any
    direction of the second body and along rigid motions of the frame owner,
    away from rest (the A-linearised rotation term is exact along rigid
    motions);
  * solves: brute-force LAPACK LU of the full KKT matrix (Eq. kkt with the
    footnote's -C) on small trees and chains mixing every joint type,
    world-tied ones included;
  * dynamics: a box on a vertical prismatic slider falls freely (the discrete
    implicit-Euler free fall in closed form), and a universal-joint pendulum
    swinging about the first axis converges to Eq. elliptic at first order.
"""
import math

import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from test_oracle_pins import (A_of, brute_force_kkt, elliptic_theta, rot)

H = 1e-2


def joint_pair(jtype, axis, axis2=None, ell=0.1, seed=0):
    """Two free boxes joined at the +x end of the first / -x end of the
    second, tilted and shifted so that nothing is axis-aligned."""
    asm = mi.chain(2, seed=seed, pin_first=False)
    Q = rot([0.3, -0.5, 0.8], 0.7)
    for b in range(2):
        for c in range(4):
            asm.q0[b, 3 * c:3 * c + 3] = Q @ asm.q0[b, 3 * c:3 * c + 3]
    asm.jtype = np.array([jtype], np.uint8)
    asm.axis = np.array([axis], float) / np.linalg.norm(axis)
    asm.axis2 = np.array([axis2 if axis2 is not None else mi.perpendicular(asm.axis)[0]], float)
    asm.cp_len = np.array([ell])
    return asm


def world_point(asm, b, p):
    return A_of(asm.q0[b]) @ p + asm.q0[b, 9:]


def rigid(q, b, R, centre):
    """Body b of state q moved by the rotation R about the world point centre."""
    out = q.copy()
    out[b, :9] = (R @ A_of(q[b])).T.reshape(9)
    out[b, 9:] = centre + R @ (q[b, 9:] - centre)
    return out


def values(s, q, k=0):
    return s.joint_terms(q, k)[0]


def test_universal_kinematics():
    a1 = np.array([0.2, 1.0, -0.3])
    a2 = mi.perpendicular(a1 / np.linalg.norm(a1))[0]
    asm = joint_pair(mi.UNIVERSAL, a1, a2)
    s = oracle.System(asm)
    q = asm.q0.copy()
    assert np.abs(values(s, q)).max() < 1e-14
    centre = world_point(asm, 0, asm.pa[0])
    R0 = A_of(q[0])  # rotation of both boxes at rest
    w1 = R0 @ (a1 / np.linalg.norm(a1))
    w2 = R0 @ a2
    # rotations of the second box about either axis through the centre: free
    for w in (w1, w2):
        for ang in (0.3, -1.1):
            assert np.abs(values(s, rigid(q, 1, rot(w, ang), centre))).max() < 1e-13
    # about the third direction: the fourth row, and only it, moves
    C = values(s, rigid(q, 1, rot(np.cross(w1, w2), 0.2), centre))
    assert np.abs(C[:3]).max() < 1e-13 and abs(C[3]) > 1e-3
    # any relative translation opens the ball rows
    qt = q.copy(); qt[1, 9:] += [1e-3, -2e-3, 5e-4]
    assert np.abs(values(s, qt)[:3]).max() > 1e-4


def test_prismatic_kinematics():
    ax = np.array([0.4, -0.2, 1.0])
    asm = joint_pair(mi.PRISMATIC, ax)
    s = oracle.System(asm)
    q = asm.q0.copy()
    assert np.abs(values(s, q)).max() < 1e-14
    w = A_of(q[0]) @ (ax / np.linalg.norm(ax))
    # sliding along the axis: free
    for d in (0.3, -0.05):
        qs = q.copy(); qs[1, 9:] += d * w
        assert np.abs(values(s, qs)).max() < 1e-13
    p1 = world_point(asm, 1, asm.pb[0])
    # a turn about the axis: only the fifth row
    C = values(s, rigid(q, 1, rot(w, 0.1), p1))
    assert np.abs(C[:4]).max() < 1e-13 and abs(C[4]) > 1e-3
    # a tilt of the axis: the third and fourth rows
    n = mi.perpendicular(w)[0]
    C = values(s, rigid(q, 1, rot(n, 0.1), p1))
    assert np.abs(C[:2]).max() < 1e-13 and np.abs(C[2:4]).max() > 1e-3
    # a sideways shift: the first two rows
    qs = q.copy(); qs[1, 9:] += 1e-3 * n
    C = values(s, qs)
    assert np.abs(C[:2]).max() > 1e-4 and np.abs(C[2:]).max() < 1e-13


@pytest.mark.parametrize("jtype", [mi.HINGE, mi.UNIVERSAL, mi.PRISMATIC])
def test_gradient_away_from_rest(jtype):
    """Central differences of C along every direction of the second body and
    along rigid motions of the frame owner (rotations about three axes through
    its centre, translations), with the joint pulled apart: both boxes turned
    and the second shifted, so that every row is far from zero (the rotation
    term is exact along rigid motions of a rotated, undeformed owner)."""
    asm = joint_pair(jtype, [0.3, 0.9, 0.2], seed=3)
    s = oracle.System(asm)
    q = rigid(asm.q0, 0, rot([1.0, -0.4, 0.2], 0.3), asm.q0[0, 9:])
    q = rigid(q, 1, rot([0.1, 0.7, -0.5], 0.2), world_point(asm, 1, asm.pb[0]))
    q[1, 9:] += [2e-3, -1e-3, 3e-3]
    C, Ga, Gb = s.joint_terms(q, 0)
    assert np.abs(C).min() > 1e-5  # not at rest
    e = 1e-6
    for j in range(12):
        qp = q.copy(); qp[1, j] += e
        qm = q.copy(); qm[1, j] -= e
        fd = (values(s, qp) - values(s, qm)) / (2 * e)
        assert np.allclose(Gb[:, j], fd, atol=1e-8), (j, Gb[:, j], fd)
    c0 = q[0, 9:].copy()
    for w in np.eye(3):
        fd = (values(s, rigid(q, 0, rot(w, e), c0)) - values(s, rigid(q, 0, rot(w, -e), c0))) / (2 * e)
        dq = np.zeros(12)
        for c in range(3):
            dq[3 * c:3 * c + 3] = np.cross(w, A_of(q[0])[:, c])
        assert np.allclose(Ga @ dq, fd, atol=1e-8), (w, Ga @ dq, fd)
        qp = q.copy(); qp[0, 9:] += e * w
        qm = q.copy(); qm[0, 9:] -= e * w
        fd = (values(s, qp) - values(s, qm)) / (2 * e)
        assert np.allclose(Ga[:, 9:] @ w, fd, atol=1e-8)


def mixed_assemblies():
    t = mi.mix_joint_types(mi.tree(14, seed=31, window=4), seed=32)
    t.qd0[1:] = np.random.default_rng(33).normal(0, 0.05, (13, 12))
    # a free chain of universal and prismatic joints hung from the world by a
    # world-owned prismatic joint at its first body, and a free chain whose
    # tip owns a universal joint to the world
    c = mi.mix_joint_types(mi.chain(6, seed=34, pin_first=False), seed=35, probs=(0.0, 0.0, 0.5, 0.5))
    p0 = c.q0[0, 9:] + np.array([0.0, 0.05, 0.0])
    c.jtype = np.append(c.jtype, mi.PRISMATIC).astype(np.uint8)
    c.ja = np.append(c.ja, -1).astype(np.int32); c.jb = np.append(c.jb, 0).astype(np.int32)
    c.pa = np.vstack([c.pa, p0]); c.pb = np.vstack([c.pb, [0.0, 0.05, 0.0]])
    c.axis = np.vstack([c.axis, [0.0, 0.6, 0.8]]); c.axis2 = np.vstack([c.axis2, [1, 0, 0]])
    c.cp_len = np.append(c.cp_len, 0.1)
    u = mi.mix_joint_types(mi.chain(4, seed=37, pin_first=False, origin=(0.0, 3.0, 0.0)), seed=38,
                           probs=(0.0, 0.0, 1.0, 0.0))
    tip = u.q0[3, 9:] + np.array([0.5, 0, 0])
    u.jtype = np.append(u.jtype, mi.UNIVERSAL).astype(np.uint8)
    u.ja = np.append(u.ja, 3).astype(np.int32); u.jb = np.append(u.jb, -1).astype(np.int32)
    u.pa = np.vstack([u.pa, [0.5, 0, 0]]); u.pb = np.vstack([u.pb, tip])
    u.axis = np.vstack([u.axis, [0, 1, 0]]); u.axis2 = np.vstack([u.axis2, [0, 0, 1]])
    u.cp_len = np.append(u.cp_len, 0.1)
    cu = mi.concat([c, u], h=H, steps=3)
    cu.qd0[:] = np.random.default_rng(36).normal(0, 0.05, cu.qd0.shape)
    return [("mixed_tree", t), ("universal_prismatic_chains", cu)]


@pytest.mark.parametrize("name,asm", mixed_assemblies(), ids=lambda x: x if isinstance(x, str) else "")
def test_mixed_joints_match_dense_kkt_lu(name, asm):
    s = oracle.System(asm)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for _ in range(3):
        dq, lam_bf = brute_force_kkt(asm, s, q, qd, asm.h)
        for sol in (oracle.TREE, oracle.DENSE):
            q1, qd1, lam, d = s.step(asm.h, q, qd, solver=sol)
            dyn = asm.pinned == 0
            scale = np.abs(dq).max()
            # the full KKT matrix of these assemblies has condition ~5e13 (the
            # dual ~1e3), so the LAPACK reference itself carries ~1e-11 of
            # rounding; the oracle's dual solves agree with it to that level
            tol = 2e-11 if sol == oracle.DENSE else 5e-11
            assert np.abs((qd1 * asm.h - dq)[dyn]).max() <= tol * scale
            assert np.abs(lam - lam_bf).max() <= 1e-10 * np.abs(lam_bf).max()
            assert d[oracle.KKT] < 1e-10
        q, qd = q1, qd1


def test_vertical_slider_falls_freely():
    """A box on a vertical prismatic joint to the world: the joint permits
    exactly the fall, so the box follows the closed-form discrete free fall
    and keeps its orientation."""
    body = mi.free_body(dims=(0.2, 0.3, 0.4), t=(1.0, 2.0, 3.0))
    body.jtype = np.array([mi.PRISMATIC], np.uint8)
    body.ja = np.array([-1], np.int32); body.jb = np.array([0], np.int32)
    body.pa = np.array([[1.0, 2.0, 3.2]]); body.pb = np.array([[0.0, 0.0, 0.2]])
    body.axis = np.array([[0.0, 0.0, 1.0]]); body.axis2 = np.array([[1.0, 0.0, 0.0]])
    body.cp_len = np.array([0.1])
    s = oracle.System(body)
    q, qd = body.q0.copy(), body.qd0.copy()
    for n in range(1, 31):
        q, qd, lam, d = s.step(H, q, qd)
        z = 3.0 - 0.5 * n * (n + 1) * H * H * 9.8
        assert abs(q[0, 11] - z) <= 1e-12 * 3.0
        assert np.abs(q[0, 9:11] - [1.0, 2.0]).max() <= 1e-13
        assert np.abs(q[0, :9] - np.eye(3).reshape(9)).max() <= 1e-12
        assert np.abs(lam).max() <= 1e-9 * 9.8 * body.density[0] * 0.024


def universal_pendulum(h, T):
    """The box of the hinge pendulum (1.0 x 0.1 x 0.1 m, pivot at its -x end,
    released horizontal) on a universal joint whose first axis is the
    horizontal y axis and second the box's long axis."""
    body = mi.free_body(dims=(1.0, 0.1, 0.1), t=(0.5, 0.0, 0.0), h=h)
    body.jtype = np.array([mi.UNIVERSAL], np.uint8)
    body.ja = np.array([-1], np.int32); body.jb = np.array([0], np.int32)
    body.pa = np.array([[0.0, 0.0, 0.0]]); body.pb = np.array([[-0.5, 0.0, 0.0]])
    body.axis = np.array([[0.0, 1.0, 0.0]]); body.axis2 = np.array([[1.0, 0.0, 0.0]])
    body.cp_len = np.array([0.1])
    s = oracle.System(body)
    q, qd = body.q0.copy(), body.qd0.copy()
    ts, th = [0.0], [0.0]
    for n in range(int(round(T / h))):
        q, qd, lam, d = s.step(h, q, qd)
        c = q[0, 9:]
        ts.append((n + 1) * h)
        th.append(math.atan2(-c[2], c[0]))
        assert abs(c[1]) < 1e-9
    return np.array(ts), np.array(th), body


def test_universal_pendulum_converges_to_elliptic_solution():
    errs = []
    for h in (4e-3, 2e-3, 1e-3):
        t, th, body = universal_pendulum(h, 0.6)
        errs.append(np.abs(th - elliptic_theta(t, body)).max())
    assert errs[0] > errs[1] > errs[2]
    order = math.log(errs[0] / errs[2]) / math.log(4.0)
    assert 0.7 < order < 1.3
    assert errs[2] < 0.02
