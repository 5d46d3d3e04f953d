"""Pins of the FP64 oracle to facts the paper and mathematics fix.

Each test states what it pins.  None of them retypes the oracle's formulas:
they use closed-form solutions, invariants, brute-force dense linear algebra
(LAPACK through numpy) and the elliptic-integral pendulum of Sec. 6.1
(Eq. elliptic).
"""
import math

import numpy as np
import pytest

import mabd_inputs as mi
import oracle

H = 1e-2


def rot(axis, ang):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def A_of(q):
    return q[0:9].reshape(3, 3).T  # columns a1, a2, a3


# --------------------------------------------------------------- single body

def test_free_fall_closed_form():
    """Implicit Euler of an unjointed rigid box under gravity (Eq. variation_energy):
    t_n = t0 + n h v0 + n(n+1)/2 h^2 g, v_n = v0 + n h g, A constant."""
    A0 = rot([1, 2, 3], 0.7)
    v0 = np.array([0.3, -1.0, 2.0])
    qd = np.zeros(12); qd[9:] = v0
    body = mi.free_body(dims=(0.3, 0.2, 0.1), A=A0, t=(1.0, 2.0, 3.0), qd=qd)
    s = oracle.System(body)
    q, qdd = body.q0.copy(), body.qd0.copy()
    g = np.array(mi.GRAVITY)
    for n in range(1, 31):
        q, qdd, _, _ = s.step(H, q, qdd)
        t_exact = np.array([1.0, 2.0, 3.0]) + n * H * v0 + 0.5 * n * (n + 1) * H * H * g
        assert np.allclose(q[0, 9:], t_exact, rtol=0, atol=1e-13)
        assert np.allclose(qdd[0, 9:], v0 + n * H * g, rtol=0, atol=1e-13)
        assert np.allclose(A_of(q[0]), A0, rtol=0, atol=1e-14)
        assert np.allclose(qdd[0, :9], 0.0, atol=1e-12)


def test_wrench_force_closed_form():
    """A force f at the COM of an unjointed box (wrench [0; f], Eq.
    module1-wrench-map) adds f / m to gravity in the implicit Euler closed form
    of test_free_fall_closed_form, and turns nothing."""
    A0 = rot([2, -1, 1], 0.4)
    v0 = np.array([0.5, 0.2, -0.3])
    qd = np.zeros(12); qd[9:] = v0
    dims = (0.3, 0.2, 0.1)
    body = mi.free_body(dims=dims, A=A0, t=(0.0, 1.0, 2.0), qd=qd)
    f = np.array([3.0, -7.0, 11.0])
    m = 1000.0 * np.prod(dims)
    s = oracle.System(body, wrench=np.concatenate([np.zeros(3), f])[None, :])
    q, qdd = body.q0.copy(), body.qd0.copy()
    acc = np.array(mi.GRAVITY) + f / m
    for n in range(1, 21):
        q, qdd, _, _ = s.step(H, q, qdd)
        assert np.allclose(q[0, 9:], np.array([0.0, 1.0, 2.0]) + n * H * v0 + 0.5 * n * (n + 1) * H * H * acc,
                           rtol=0, atol=1e-13)
        assert np.allclose(qdd[0, 9:], v0 + n * H * acc, rtol=0, atol=1e-12)
        assert np.allclose(A_of(q[0]), A0, rtol=0, atol=1e-14)


def test_wrench_torque_spins_cube_rigidly():
    """A torque tau on a cube at rest (any orientation R0, no gravity): the
    affine increment is R0-skew, so the stiff stretch modes stay idle and one
    implicit Euler step gives the rigid answer omega = h tau / I with
    I = m a^2 / 6, read through the twist map omega = 1/2 sum_c q_c x qdot_c
    (Eq. module1-omega-v)."""
    a = 0.2
    for R0 in (np.eye(3), rot([1, 1, 0], 0.9)):
        body = mi.free_body(dims=(a, a, a), A=R0, t=(0.0, 0.0, 1.0))
        tau = np.array([0.4, -1.2, 2.5])
        s = oracle.System(body, gravity=(0.0, 0.0, 0.0), wrench=np.concatenate([tau, np.zeros(3)])[None, :])
        q1, qd1, _, _ = s.step(H, body.q0, body.qd0)
        A1, Ad = A_of(q1[0]), qd1[0, 0:9].reshape(3, 3).T
        omega = 0.5 * sum(np.cross(A1[:, c] - H * Ad[:, c], Ad[:, c]) for c in range(3))
        inertia = 1000.0 * a ** 3 * a * a / 6.0
        # the 12x12 solve mixes the skew direction (inertia only) with the
        # stiff stretch modes: kappa(Hbar) ~ 1e4, so ~1e-12 of rounding
        assert np.allclose(omega, H * tau / inertia, rtol=1e-10, atol=0)
        assert np.allclose(qd1[0, 9:], 0.0, atol=1e-15)


def test_wrench_map_is_power_consistent():
    """Virtual work: the affine force of a wrench satisfies f_A,ext . qdot =
    tau . omega + f . v for every velocity, with omega, v from the twist map
    (Eqs. module1-G-twist, module1-omega-v).  f_A,ext is read from the oracle
    as the difference of its forces with and without the wrench, at a
    deformed, rotated configuration (a soft body at rest, so that the other
    force terms are small and the difference is exact to rounding)."""
    rng = np.random.default_rng(3)
    A0 = rot([0.3, 1, -2], 1.1) @ (np.eye(3) + 0.05 * rng.normal(size=(3, 3)))
    body = mi.free_body(dims=(0.3, 0.25, 0.15), A=A0, t=(1.0, -2.0, 0.5), k_orth=1.0)
    W = rng.normal(size=6)
    q = body.q0.copy()
    qd0 = np.zeros((1, 12))
    _, f0, _ = oracle.System(body).body_terms(H, q, qd0, 0)
    _, fw, _ = oracle.System(body, wrench=W[None, :]).body_terms(H, q, qd0, 0)
    fext = fw - f0
    for _ in range(5):
        v = rng.normal(size=12)
        omega = 0.5 * sum(np.cross(q[0, 3 * c:3 * c + 3], v[3 * c:3 * c + 3]) for c in range(3))
        assert abs(fext @ v - (W[:3] @ omega + W[3:] @ v[9:])) <= 1e-12 * (1 + abs(fext @ v))


@pytest.mark.parametrize("material,E,nu", [(0, 1e6, 0.0), (1, 1e6, 0.3)])
def test_stretch_mode_is_implicit_euler_oscillator(material, E, nu):
    """A box stretched along its own x axis keeps R = I (polar of a symmetric
    positive matrix), so that mode is a linear oscillator with stiffness
    V (2 mu + lambda) and mass m lx^2 / 12 (Sec. 3.3, linear elasticity).
    Implicit Euler maps (x, v) by the matrix [[1, h], [-h w^2, 1]] / (1 + h^2 w^2).
    With lambda != 0 the three diagonal entries couple; the closed form below
    uses the exact 3-mode decomposition of that coupling."""
    dims = np.array([0.4, 0.2, 0.1])
    rho = 800.0
    eps = 1e-3
    A0 = np.diag([1 + eps, 1.0, 1.0])
    body = mi.free_body(dims=dims, density=rho, k_orth=E, A=A0)
    body.material = material
    body.poisson = np.array([nu])
    body.gravity = (0.0, 0.0, 0.0)
    s = oracle.System(body)
    V = dims.prod(); m = rho * V
    if material == 0:
        mu, lam = 4 * E, 0.0
    else:
        mu, lam = E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))
    Mi = m * dims ** 2 / 12.0                       # mass of each diagonal entry
    Kd = V * (2 * mu * np.eye(3) + lam * np.ones((3, 3)))  # stiffness on (A00, A11, A22)
    # implicit Euler on M x'' = -K x: (M/h^2 + K) x1 = M/h^2 (x0 + h v0), v1 = (x1 - x0)/h
    Mm = np.diag(Mi)
    x = np.array([eps, 0.0, 0.0]); v = np.zeros(3)
    q, qd = body.q0.copy(), body.qd0.copy()
    for _ in range(20):
        x1 = np.linalg.solve(Mm / H ** 2 + Kd, Mm / H ** 2 @ (x + H * v))
        v = (x1 - x) / H
        x = x1
        q, qd, _, _ = s.step(H, q, qd)
        diag = np.array([q[0, 0], q[0, 4], q[0, 8]]) - 1.0
        assert np.allclose(diag, x, rtol=0, atol=1e-14 + 1e-10 * eps)
        assert np.allclose([qd[0, 0], qd[0, 4], qd[0, 8]], v, rtol=0, atol=1e-10 * eps / H)
        off = q[0, [1, 2, 3, 5, 6, 7]]
        assert np.abs(off).max() < 1e-15


def test_rotation_equivariance_single_and_chain():
    """Co-rotation (Eq. abd_r): rotating the whole scene by Q (state, gravity and
    world anchors) rotates the step's result by diag4(Q)."""
    Q = rot([0.3, -1.0, 0.5], 1.1)
    for asm in (mi.chain(6, seed=2, hinge_frac=0.5), mi.tree(9, seed=4)):
        asm.qd0[:, :] = np.random.default_rng(0).normal(0, 0.1, asm.qd0.shape)
        asm.qd0[asm.pinned == 1] = 0.0
        s1 = oracle.System(asm)
        q1, qd1, lam1, _ = s1.step(H, asm.q0, asm.qd0)
        r = asm.copy()
        for b in range(r.n):
            for c in range(4):
                r.q0[b, 3 * c:3 * c + 3] = Q @ asm.q0[b, 3 * c:3 * c + 3]
                r.qd0[b, 3 * c:3 * c + 3] = Q @ asm.qd0[b, 3 * c:3 * c + 3]
        r.gravity = tuple(Q @ np.array(asm.gravity))
        s2 = oracle.System(r)
        q2, qd2, lam2, _ = s2.step(H, r.q0, r.qd0)
        for b in range(asm.n):
            for c in range(4):
                assert np.allclose(q2[b, 3 * c:3 * c + 3], Q @ q1[b, 3 * c:3 * c + 3],
                                   rtol=0, atol=1e-13 * max(1.0, np.abs(q1[b]).max()))
                assert np.allclose(qd2[b, 3 * c:3 * c + 3], Q @ qd1[b, 3 * c:3 * c + 3],
                                   rtol=0, atol=1e-10 * max(1e-3, np.abs(qd1).max()))


def affine_momenta(asm, q, qd):
    """Linear and angular momentum of affine boxes: p = m tdot,
    L = m t x tdot + sum_c Mbar_c a_c x adot_c (integral of rho x cross xdot)."""
    V = asm.dims.prod(axis=1); m = asm.density * V
    Mb = m[:, None] * asm.dims ** 2 / 12.0
    p = (m[:, None] * qd[:, 9:]).sum(0)
    L = np.zeros(3)
    for b in range(asm.n):
        L += m[b] * np.cross(q[b, 9:], qd[b, 9:])
        for c in range(3):
            L += Mb[b, c] * np.cross(q[b, 3 * c:3 * c + 3], qd[b, 3 * c:3 * c + 3])
    return p, L


def spinning_box(h, omega=None, v=None, dims=(0.1, 0.1, 0.1)):
    """Sec. 6.1 spinning box: 0.1 m cube, rho 1e3, E 1e9, nu 0.3, p0 = (100,0,0),
    L0 = (0,100,0); the spin enters through qdot = E(A) V (Eq. module2-E)."""
    dims = np.asarray(dims, float); rho = 1e3
    m = rho * dims.prod(); I = m * (dims[0] ** 2 + dims[2] ** 2) / 12.0
    omega = np.array([0.0, 100.0 / I, 0.0]) if omega is None else np.asarray(omega, float)
    v = np.array([100.0 / m, 0.0, 0.0]) if v is None else np.asarray(v, float)
    qd = np.zeros(12)
    A = np.eye(3)
    for c in range(3):
        qd[3 * c:3 * c + 3] = np.cross(omega, A[:, c])
    qd[9:] = v
    b = mi.free_body(dims=dims, density=rho, k_orth=1e9, qd=qd, h=h)
    b.material = 1; b.poisson = np.array([0.3]); b.gravity = (0.0, 0.0, 0.0)
    return b


def energy(b, q, qd):
    """Kinetic energy 1/2 qdot^T M_A qdot plus co-rotated linear elastic energy."""
    V = b.dims.prod(axis=1)[0]; m = b.density[0] * V; Mb = m * b.dims[0] ** 2 / 12.0
    E, nu = b.k_orth[0], b.poisson[0]
    mu, lam = E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))
    ke = 0.5 * m * qd[0, 9:] @ qd[0, 9:] + 0.5 * sum(Mb[c] * qd[0, 3 * c:3 * c + 3] @ qd[0, 3 * c:3 * c + 3] for c in range(3))
    A = A_of(q[0]); U, S, Vt = np.linalg.svd(A); R = U @ Vt
    e = 0.5 * (R.T @ A + A.T @ R) - np.eye(3)
    return ke + V * (mu * (e * e).sum() + 0.5 * lam * np.trace(e) ** 2), S


def test_spinning_box_linear_momentum():
    """Linear momentum of the paper's spinning cube is preserved at all h (Sec. 6.1)."""
    for h in (1e-2, 5e-3, 2.5e-3):
        b = spinning_box(h)
        s = oracle.System(b)
        q, qd = b.q0.copy(), b.qd0.copy()
        p0, L0 = affine_momenta(b, q, qd)
        assert np.allclose(p0, [100.0, 0, 0]) and np.allclose(L0, [0, 100.0, 0], rtol=1e-12)
        for _ in range(int(round(0.2 / h))):
            q, qd, _, _ = s.step(h, q, qd)
            p, L = affine_momenta(b, q, qd)
            assert np.allclose(p, p0, rtol=1e-13, atol=1e-11)


def test_tumbling_box_converges_with_h():
    """A box tumbling about a non-principal axis: linear momentum is exact, the
    angular-momentum drift shrinks as h shrinks (Sec. 6.1), one Newton iteration
    leaves a stretch of order (omega h)^2 (the linearisation error of Eq. newton),
    and converged Newton iterations make implicit Euler dissipate energy, less
    for smaller h."""
    drift, stretch, loss = {}, {}, {}
    for h in (1e-2, 5e-3, 2.5e-3):
        for iters in (1, 4):
            b = spinning_box(h, omega=[1.0, 8.0, 2.0], v=[1.0, 0.0, 0.0], dims=(0.3, 0.2, 0.1))
            s = oracle.System(b, newton_iters=iters)
            q, qd = b.q0.copy(), b.qd0.copy()
            p0, L0 = affine_momenta(b, q, qd)
            E0, _ = energy(b, q, qd)
            for _ in range(int(round(1.0 / h))):
                q, qd, _, _ = s.step(h, q, qd)
            p, L = affine_momenta(b, q, qd)
            assert np.allclose(p, p0, rtol=1e-12, atol=1e-12)
            E1, S = energy(b, q, qd)
            if iters == 1:
                drift[h] = abs(1.0 - np.linalg.norm(L) / np.linalg.norm(L0))
                stretch[h] = S.max() - 1.0
            else:
                loss[h] = 1.0 - E1 / E0
    assert drift[1e-2] > drift[5e-3] > drift[2.5e-3]
    assert 10.0 < stretch[1e-2] / stretch[2.5e-3] < 22.0
    assert loss[1e-2] > loss[5e-3] > loss[2.5e-3] > 0.0


def test_polar_against_svd():
    """Eq. polar: R = U V^T from the SVD A = U S V^T (det A > 0)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        A = rot(rng.normal(size=3), rng.uniform(0, 3)) @ (np.eye(3) + 0.3 * rng.normal(size=(3, 3)))
        if np.linalg.det(A) <= 0:
            continue
        U, S, Vt = np.linalg.svd(A)
        assert np.allclose(oracle.polar(A), U @ Vt, atol=1e-13)
    with pytest.raises(oracle.OracleError):
        oracle.polar(np.diag([1.0, 1.0, -1.0]))


# ------------------------------------------------------------ joint systems

def kkt_matrix(asm, s, q, qd, h):
    """The full KKT matrix of Eq. kkt and its right-hand side [f; -C] (the
    footnote's -C), assembled from the oracle's per-body H, f and per-joint
    C, G.  Returns (K, rhs, col, nq): col maps a dynamic body to its first
    column, nq is the number of primal unknowns."""
    dyn = [i for i in range(asm.n) if not asm.pinned[i]]
    col = {b: 12 * k for k, b in enumerate(dyn)}
    nq = 12 * len(dyn)
    rows = [mi.JOINT_ROWS[t] for t in asm.jtype]
    nl = sum(rows)
    K = np.zeros((nq + nl, nq + nl)); rhs = np.zeros(nq + nl)
    for b in dyn:
        Hb, fb, _ = s.body_terms(h, q, qd, b)
        K[col[b]:col[b] + 12, col[b]:col[b] + 12] = Hb
        rhs[col[b]:col[b] + 12] = fb
    r0 = nq
    for k in range(asm.m):
        C, Ga, Gb = s.joint_terms(q, k)
        rk = rows[k]
        for side, G in ((asm.ja[k], Ga), (asm.jb[k], Gb)):
            if side >= 0 and not asm.pinned[side]:
                K[r0:r0 + rk, col[side]:col[side] + 12] = G
                K[col[side]:col[side] + 12, r0:r0 + rk] = G.T
        rhs[r0:r0 + rk] = -C
        r0 += rk
    return K, rhs, col, nq


def brute_force_kkt(asm, s, q, qd, h):
    """Solve the full KKT of Eq. kkt (with -C on the right) with LAPACK."""
    K, rhs, col, nq = kkt_matrix(asm, s, q, qd, h)
    x = np.linalg.solve(K, rhs)
    dq = np.zeros((asm.n, 12))
    for b, c in col.items():
        dq[b] = x[c:c + 12]
    return dq, x[nq:]


def small_assemblies():
    c = mi.chain(12, seed=7, hinge_frac=0.5)
    c.qd0[1:] = np.random.default_rng(1).normal(0, 0.05, (11, 12))
    t = mi.tree(14, seed=8, window=4)
    t.qd0[1:] = np.random.default_rng(2).normal(0, 0.05, (13, 12))
    # a chain whose far end is also tied to the world by a ball joint
    w = mi.chain(8, seed=9, hinge_frac=0.5)
    w.jtype = np.append(w.jtype, 0).astype(np.uint8)
    w.ja = np.append(w.ja, 7).astype(np.int32)
    w.jb = np.append(w.jb, -1).astype(np.int32)
    tip = w.q0[7, 9:] + np.array([0.5, 0, 0])
    w.pa = np.vstack([w.pa, [0.5, 0, 0]]); w.pb = np.vstack([w.pb, tip])
    w.axis = np.vstack([w.axis, [0, 1, 0]]); w.cp_len = np.append(w.cp_len, 0.1)
    # a hinge whose frame owner is the world
    hw = mi.chain(5, seed=10, hinge_frac=1.0, pin_first=False)
    hw.jtype = np.append(hw.jtype, 1).astype(np.uint8)
    hw.ja = np.append(hw.ja, -1).astype(np.int32)
    hw.jb = np.append(hw.jb, 0).astype(np.int32)
    p0 = hw.q0[0, 9:] - np.array([0.5, 0, 0])
    hw.pa = np.vstack([hw.pa, p0]); hw.pb = np.vstack([hw.pb, [-0.5, 0, 0]])
    hw.axis = np.vstack([hw.axis, [0.0, 0.6, 0.8]]); hw.cp_len = np.append(hw.cp_len, 0.1)
    return [("chain", c, oracle.CHAIN), ("tree", t, oracle.TREE), ("chain_world", w, oracle.TREE),
            ("hinge_world", hw, oracle.TREE)]


@pytest.mark.parametrize("name,asm,solver", small_assemblies(), ids=lambda x: x if isinstance(x, str) else "")
def test_solvers_match_dense_kkt_lu(name, asm, solver):
    """Chain (block Thomas) and tree (condensation) solves equal the LAPACK
    solution of the full KKT system (Eq. kkt with the footnote's -C)."""
    s = oracle.System(asm)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for _ in range(3):
        dq, lam_bf = brute_force_kkt(asm, s, q, qd, asm.h)
        for sol in (solver, oracle.DENSE):
            q1, qd1, lam, d = s.step(asm.h, q, qd, solver=sol)
            scale = np.abs(dq).max()
            dyn = asm.pinned == 0
            # the primal condensation accumulates G^T S^-1 G into 12x12 blocks whose
            # conditioning grows along a branch; the dual dense solve does not
            tol = 5e-12 if sol == oracle.DENSE else 3e-11
            assert np.abs((qd1 * asm.h - dq)[dyn]).max() <= tol * scale
            assert np.abs((q1 - q)[dyn] - dq[dyn]).max() <= tol * scale + 4e-16 * np.abs(q).max()
            assert np.abs(lam - lam_bf).max() <= 1e-10 * np.abs(lam_bf).max()
            assert d[oracle.KKT] < 1e-10
        q, qd = q1, qd1


def test_chain_equals_tree_solver():
    """A path fed to the tree condensation gives the chain (Thomas) result."""
    asm = mi.chain(40, seed=11, hinge_frac=0.5)
    s = oracle.System(asm)
    a = s.step(asm.h, asm.q0, asm.qd0, solver=oracle.CHAIN)
    b = s.step(asm.h, asm.q0, asm.qd0, solver=oracle.TREE)
    assert np.abs(a[0] - b[0]).max() < 1e-13 * np.abs(a[0]).max()
    assert np.abs(a[1] - b[1]).max() < 1e-10 * np.abs(a[1]).max()


def test_ball_constraints_exact_every_step():
    """With the -C term (footnote of Eq. kkt) ball joints are linear in q, so a
    direct dual solve leaves them satisfied to rounding after every step."""
    asm = mi.chain(64, seed=0)
    s = oracle.System(asm)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for _ in range(50):
        q, qd, lam, d = s.step(asm.h, q, qd)
        assert d[oracle.CBALL] < 1e-13 * max(1.0, np.abs(q[:, 9:]).max())
        assert d[oracle.KKT] < 1e-11


def test_dual_matrix_structure():
    """S = G H^-1 G^T is symmetric positive definite and block-sparse: a block
    (k, l) is nonzero only if joints k and l share a dynamic body (Fig. dual_mat)."""
    asm = mi.tree(30, seed=12, window=5)
    s = oracle.System(asm)
    S, r = s.dual(asm.h, asm.q0, asm.qd0)
    S = S.toarray()
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    np.linalg.cholesky(S)
    rows = [mi.JOINT_ROWS[t] for t in asm.jtype]
    off = np.concatenate([[0], np.cumsum(rows)])
    for k in range(asm.m):
        for l in range(asm.m):
            bk = {asm.ja[k], asm.jb[k]} - {-1}; bl = {asm.ja[l], asm.jb[l]} - {-1}
            shared = [b for b in bk & bl if not asm.pinned[b]]
            blk = S[off[k]:off[k + 1], off[l]:off[l + 1]]
            if not shared:
                assert np.all(blk == 0.0)
            else:
                assert np.abs(blk).max() > 0.0


def test_pcg_matches_direct_on_small_lattice():
    asm = mi.lattice(6, seed=3)
    s = oracle.System(asm)
    assert s.classify() == 3
    a = s.step(asm.h, asm.q0, asm.qd0, solver=oracle.DENSE)
    b = s.step(asm.h, asm.q0, asm.qd0, solver=oracle.PCG, tol=1e-13, max_iters=20000)
    c = s.step_sparse(asm.h, asm.q0, asm.qd0)
    assert b[3][oracle.RHO_D] <= 1e-12
    assert np.abs(a[2] - b[2]).max() < 1e-7 * np.abs(a[2]).max()
    assert np.abs(a[2] - c[2]).max() < 1e-9 * np.abs(a[2]).max()
    assert np.abs(a[0] - b[0]).max() < 1e-12 * np.abs(a[0]).max()


def test_hinge_gradient_finite_difference_at_rest():
    """At a configuration where both control-point pairs coincide (d_m = 0), the
    hinge gradient is the plain derivative of its constraint value: compare
    the oracle's G with central differences of its own C (Eq. constraint_gradient)."""
    asm = mi.chain(3, seed=13, hinge_frac=1.0, sigma=0.0, pin_first=False)
    Q = rot([1, 1, 0], 0.4)
    for b in range(asm.n):
        for c in range(4):
            asm.q0[b, 3 * c:3 * c + 3] = Q @ asm.q0[b, 3 * c:3 * c + 3]
    s = oracle.System(asm)
    q = asm.q0.copy()
    for k in range(asm.m):
        C, Ga, Gb = s.joint_terms(q, k)
        assert np.abs(C).max() < 1e-14
        for side, G in ((asm.ja[k], Ga), (asm.jb[k], Gb)):
            for j in range(12):
                e = 1e-6
                qp = q.copy(); qp[side, j] += e
                qm = q.copy(); qm[side, j] -= e
                fd = (s.joint_terms(qp, k)[0] - s.joint_terms(qm, k)[0]) / (2 * e)
                assert np.allclose(G[:, j], fd, atol=1e-8)


def test_hinge_second_point_rows_are_normal_to_the_axis():
    """The hinge's two rows on the second control-point pair constrain only
    the directions normal to the hinge axis (Sec. 4.3: the frame maps the axis
    onto one coordinate and keeps the other two).  Stretching the hinged body
    along the axis about the first control point moves the second one along
    the axis only: no row of C may change.  A shear that moves the second
    point normal to the axis must change those two rows (the check is not
    vacuous)."""
    asm = pins_world_hinge()
    s = oracle.System(asm)
    k, b = asm.m - 1, 0
    a = asm.axis[k] / np.linalg.norm(asm.axis[k])
    q = asm.q0.copy()
    cp1 = A_of(q[b]) @ asm.pb[k] + q[b, 9:]

    def stretched(direction, eps):
        # x -> cp1 + (I + eps direction a^T)(x - cp1): cp1 stays, the second
        # control point (on the axis through cp1) moves along `direction`
        S = np.eye(3) + eps * np.outer(direction, a)
        qs = q.copy()
        qs[b, :9] = (S @ A_of(q[b])).T.reshape(9)
        qs[b, 9:] = cp1 + S @ (q[b, 9:] - cp1)
        return s.joint_terms(qs, k)[0]

    e = 1e-6
    dC = (stretched(a, e) - stretched(a, -e)) / (2 * e)
    assert np.abs(dC).max() < 1e-8 * asm.cp_len[k]
    n = np.cross(a, [1.0, 0.0, 0.0]); n /= np.linalg.norm(n)
    dCn = (stretched(n, e) - stretched(n, -e)) / (2 * e)
    assert np.abs(dCn[3:]).max() > 0.1 * asm.cp_len[k]


def pins_world_hinge():
    """The world-owned oblique hinge of small_assemblies()."""
    return small_assemblies()[3][1]


# ---------------------------------------------------------------- pendulum

def pendulum_run(h, T, hinge=False):
    """Box 1.0 x 0.1 x 0.1 m hanging from its -x end centre, released horizontal
    at rest under gravity; returns times and the angle below the horizontal."""
    body = mi.free_body(dims=(1.0, 0.1, 0.1), t=(0.5, 0.0, 0.0), h=h)
    body.jtype = np.array([1 if hinge else 0], np.uint8)
    body.ja = np.array([0], np.int32); body.jb = np.array([-1], np.int32)
    body.pa = np.array([[-0.5, 0.0, 0.0]]); body.pb = np.array([[0.0, 0.0, 0.0]])
    body.axis = np.array([[0.0, 1.0, 0.0]]); body.cp_len = np.array([0.1])
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


def elliptic_theta(t, body):
    """Eq. elliptic with kappa = sin(pi/4) (release from the horizontal) and
    omega_lin = sqrt(m g d / I_pivot); scipy's ellipj/ellipk take m = kappa^2."""
    from scipy.special import ellipj, ellipk

    lx, ly, lz = body.dims[0]
    m = body.density[0] * lx * ly * lz
    d = 0.5 * lx
    I = m * (lx ** 2 + lz ** 2) / 12.0 + m * d * d
    w = math.sqrt(m * 9.8 * d / I)
    kap = math.sin(math.pi / 4)
    sn = ellipj(ellipk(kap ** 2) - w * t, kap ** 2)[0]
    return math.pi / 2 - 2 * np.arcsin(kap * sn)


@pytest.mark.parametrize("hinge", [False, True])
def test_pendulum_converges_to_elliptic_solution(hinge):
    """Sec. 6.1 physical pendulum: theta(t) approaches Eq. elliptic as h shrinks,
    at first order in h (implicit Euler)."""
    errs = []
    for h in (4e-3, 2e-3, 1e-3):
        t, th, body = pendulum_run(h, 0.6, hinge)
        errs.append(np.abs(th - elliptic_theta(t, body)).max())
    assert errs[0] > errs[1] > errs[2]
    order = math.log(errs[0] / errs[2]) / math.log(4.0)
    assert 0.7 < order < 1.3
    assert errs[2] < 0.02


def test_hinge_blocks_off_axis_rotation():
    """A hinge with a vertical axis carries the box's weight: the tip does not
    fall beyond the elastic sag of the near-rigid body (Sec. 4.3)."""
    body = mi.free_body(dims=(1.0, 0.1, 0.1), t=(0.5, 0.0, 0.0))
    body.jtype = np.array([1], np.uint8)
    body.ja = np.array([0], np.int32); body.jb = np.array([-1], np.int32)
    body.pa = np.array([[-0.5, 0.0, 0.0]]); body.pb = np.array([[0.0, 0.0, 0.0]])
    body.axis = np.array([[0.0, 0.0, 1.0]]); body.cp_len = np.array([0.1])
    s = oracle.System(body)
    q, qd = body.q0.copy(), body.qd0.copy()
    for _ in range(100):
        q, qd, lam, d = s.step(H, q, qd)
    assert abs(q[0, 11]) < 1e-4
