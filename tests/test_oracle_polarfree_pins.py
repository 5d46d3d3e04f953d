"""Pins of the oracle's polar-free single-body solve (Alg. 1 with Eq.
len_preserving), taken by bodies without joints when body_solve = 1.

The length-preserving stand-in for a rotation is exact when A is a rotation
times a positive scale, so there the polar-free step must equal the polar
step (Eq. abd_final with Eq. polar) to rounding, forces, elastic response and
increment alike; for a general deformation it differs at first order in the
deformation, which the last pin measures."""
import numpy as np

import mabd_inputs as mi
import oracle
from test_oracle_pins import rot

H = 1e-2


def body(A, qd, k=1e7):
    b = mi.free_body(dims=(0.3, 0.2, 0.1), k_orth=k, A=A, t=(0.4, -0.2, 1.0))
    b.qd0 = np.asarray(qd, float).reshape(1, 12)
    return b


def wrench():
    return np.array([[0.3, -0.2, 0.5, 1.0, 2.0, -0.5]])


def step_pair(b, w=None):
    sp = oracle.System(b, wrench=w)
    sf = oracle.System(b, wrench=w, body_solve=1)
    a = sp.step(H, b.q0, b.qd0)
    f = sf.step(H, b.q0, b.qd0)
    return a, f


def spin_velocity(A, om, v):
    qd = np.zeros(12)
    for c in range(3):
        qd[3 * c:3 * c + 3] = np.cross(om, A[:, c])
    qd[9:] = v
    return qd


def test_equals_polar_step_for_rotations():
    rng = np.random.default_rng(5)
    for _ in range(4):
        R = rot(rng.normal(size=3), rng.uniform(0.2, 3.0))
        qd = spin_velocity(R, rng.normal(0, 3, 3), rng.normal(0, 1, 3))
        b = body(R, qd)
        for w in (None, wrench()):
            (qa, qda, _, _), (qf, qdf, _, _) = step_pair(b, w)
            assert np.abs(qf - qa).max() <= 1e-14 * np.abs(qa).max()
            assert np.abs(qdf - qda).max() <= 1e-11 * np.abs(qda).max()


def test_equals_polar_step_for_scaled_rotations():
    """A = s R: the stand-in still recovers R exactly, and the isotropic
    stretch gets the same elastic restoring force."""
    rng = np.random.default_rng(6)
    for s in (1.001, 0.998):
        R = rot(rng.normal(size=3), 1.3)
        qd = spin_velocity(R, [0.5, -1.0, 2.0], [0.1, 0.0, 0.3])
        b = body(s * R, qd)
        (qa, qda, _, _), (qf, qdf, _, _) = step_pair(b, wrench())
        assert np.abs(qf - qa).max() <= 1e-14 * np.abs(qa).max()
        assert np.abs(qdf - qda).max() <= 1e-10 * np.abs(qda).max()


def test_free_fall_closed_form():
    b = body(np.eye(3), np.zeros(12))
    s = oracle.System(b, body_solve=1)
    q, qd = b.q0.copy(), b.qd0.copy()
    for n in range(1, 21):
        q, qd, _, _ = s.step(H, q, qd)
        z = 1.0 - 0.5 * n * (n + 1) * H * H * 9.8
        assert abs(q[0, 11] - z) <= 1e-14
        assert np.abs(q[0, :9] - np.eye(3).reshape(9)).max() <= 1e-15


def test_first_order_difference_under_shear():
    """A = R (I + e N), N a fixed shear: the polar-free and polar steps differ
    at first order in e (halving e halves the difference)."""
    R = rot([0.2, 1.0, -0.4], 0.9)
    N = np.array([[0.0, 1.0, 0.3], [0.2, 0.0, -0.5], [0.7, 0.1, 0.0]])
    diffs = []
    for e in (4e-4, 2e-4, 1e-4):
        A = R @ (np.eye(3) + e * N)
        b = body(A, spin_velocity(A, [1.0, 2.0, -1.0], [0.0, 0.5, 0.0]), k=1e5)
        (qa, qda, _, _), (qf, qdf, _, _) = step_pair(b)
        diffs.append(np.abs(qdf - qda).max() / np.abs(qda).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert diffs[2] > 1e-9, diffs
    assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4, diffs


def test_jointed_bodies_keep_the_polar_solve():
    c = mi.chain(6, seed=3)
    c.qd0[1:] = np.random.default_rng(4).normal(0, 0.05, (5, 12))
    a = oracle.System(c).step(H, c.q0, c.qd0)
    f = oracle.System(c, body_solve=1).step(H, c.q0, c.qd0)
    assert np.array_equal(a[0], f[0]) and np.array_equal(a[1], f[1])
