"""Pins of the oracle's verifier: the KKT residuals and post-step constraint
values it reports for a step computed elsewhere (``System.residual``).

The verifier is the judge of every check where the oracle cannot afford the
solve itself (full-size lattices and networks, whole batches, the GPU's
device-side diagnostics), so it is pinned here against numbers that do not
come from it:

  * closed forms: with the primal equation satisfied exactly, the multipliers
    s * lambda* leave the dual residual G dq + C = (1 - s) r, so rho_d = |1 - s|
    for every assembly (r the dual right-hand side G H^-1 f + C, Eq. dual with
    the footnote's -C of Eq. kkt);
  * brute force: the residual of the full KKT matrix of Eq. kkt, formed and
    multiplied out by numpy, split into its primal rows (H dq + G^T lam - f)
    and dual rows (G dq + C);
  * plain geometry: a ball joint's post-step value is the distance of its two
    anchor points A p + t, computed here from the state.
"""
import math

import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from test_oracle_pins import brute_force_kkt, kkt_matrix


def case():
    """Mixed ball/hinge chain with a world-tied tip, mid-motion."""
    asm = mi.chain(9, seed=21, hinge_frac=0.5)
    asm.jtype = np.append(asm.jtype, 0).astype(np.uint8)
    asm.ja = np.append(asm.ja, 8).astype(np.int32)
    asm.jb = np.append(asm.jb, -1).astype(np.int32)
    tip = asm.q0[8, 9:] + np.array([0.5, 0, 0])
    asm.pa = np.vstack([asm.pa, [0.5, 0, 0]]); asm.pb = np.vstack([asm.pb, tip])
    asm.axis = np.vstack([asm.axis, [0, 1, 0]]); asm.cp_len = np.append(asm.cp_len, 0.1)
    rng = np.random.default_rng(4)
    asm.qd0[1:] = rng.normal(0, 0.05, (asm.n - 1, 12))
    s = oracle.System(asm)
    q, qd, _, _ = s.step(asm.h, asm.q0, asm.qd0)   # a state away from rest
    return asm, s, q, qd


def numpy_residuals(asm, s, q, qd, dq, lam):
    """rho_p, rho_d from the brute-force KKT matrix (numpy only)."""
    K, rhs, col, nq = kkt_matrix(asm, s, q, qd, asm.h)
    x = np.zeros(K.shape[0])
    for b, c in col.items():
        x[c:c + 12] = dq[b]
    x[nq:] = lam
    res = K @ x - rhs                 # [H dq + G^T lam - f ; G dq + C]
    hp, hf = [], []
    Ginv_f = np.zeros(K.shape[0] - nq)
    for b, c in col.items():
        Hb = K[c:c + 12, c:c + 12]
        hp.append(np.linalg.solve(Hb, res[c:c + 12]))
        y = np.linalg.solve(Hb, rhs[c:c + 12])
        hf.append(y)
        Ginv_f += K[nq:, c:c + 12] @ y
    r = Ginv_f - rhs[nq:]             # G H^-1 f + C
    rho_p = np.linalg.norm(np.concatenate(hp)) / np.linalg.norm(np.concatenate(hf))
    rho_d = np.linalg.norm(res[nq:]) / np.linalg.norm(r)
    return rho_p, rho_d


def back_projected(asm, s, q, qd, lam):
    """dq solving the primal rows exactly for given multipliers (numpy)."""
    K, rhs, col, nq = kkt_matrix(asm, s, q, qd, asm.h)
    dq = np.zeros((asm.n, 12))
    for b, c in col.items():
        dq[b] = np.linalg.solve(K[c:c + 12, c:c + 12], rhs[c:c + 12] - K[c:c + 12, nq:] @ lam)
    return dq


def test_exact_solution_has_zero_residual():
    asm, s, q, qd = case()
    dq, lam = brute_force_kkt(asm, s, q, qd, asm.h)
    d = s.residual(asm.h, q, qd, dq, lam)
    rp, rd = numpy_residuals(asm, s, q, qd, dq, lam)
    # H = diag4(R) Hbar diag4(R)^T has kappa ~ 1e5: r_p carries kappa * eps
    assert d[oracle.RHO_P] < 1e-10 and d[oracle.RHO_D] < 1e-12
    assert rp < 1e-10 and rd < 1e-12
    assert d[oracle.KKT] == max(d[oracle.RHO_P], d[oracle.RHO_D])


@pytest.mark.parametrize("scale", [0.0, 0.5, 2.0, -1.0])
def test_scaled_multipliers_give_closed_form_dual_residual(scale):
    """dq = H^-1 (f - G^T s lambda*) gives G dq + C = (1 - s) r: rho_d = |1 - s|."""
    asm, s, q, qd = case()
    _, lam = brute_force_kkt(asm, s, q, qd, asm.h)
    dq = back_projected(asm, s, q, qd, scale * lam)
    d = s.residual(asm.h, q, qd, dq, scale * lam)
    assert d[oracle.RHO_D] == pytest.approx(abs(1.0 - scale), rel=1e-9, abs=1e-11)
    assert d[oracle.RHO_P] < 1e-10


def test_perturbed_step_matches_brute_force_residual():
    """Arbitrary dq and lambda: both residuals equal the brute-force ones."""
    asm, s, q, qd = case()
    dq0, lam0 = brute_force_kkt(asm, s, q, qd, asm.h)
    rng = np.random.default_rng(5)
    for eps in (1e-8, 1e-4, 1e-1):
        dq = dq0 + eps * np.abs(dq0).max() * rng.normal(size=dq0.shape)
        dq[asm.pinned == 1] = 0.0
        lam = lam0 + eps * np.abs(lam0).max() * rng.normal(size=lam0.shape)
        d = s.residual(asm.h, q, qd, dq, lam)
        rp, rd = numpy_residuals(asm, s, q, qd, dq, lam)
        assert d[oracle.RHO_P] == pytest.approx(rp, rel=1e-7)
        assert d[oracle.RHO_D] == pytest.approx(rd, rel=1e-7)
        assert rp > 1e-9 and rd > 1e-9


def test_primal_residual_is_relative_to_the_free_increment():
    """lam exact, dq = dq* + delta on one body: H^-1 r_p = delta there and zero
    elsewhere, so rho_p = |delta| / |H^-1 f| with H^-1 f from numpy."""
    asm, s, q, qd = case()
    dq, lam = brute_force_kkt(asm, s, q, qd, asm.h)
    K, rhs, col, nq = kkt_matrix(asm, s, q, qd, asm.h)
    hf = np.concatenate([np.linalg.solve(K[c:c + 12, c:c + 12], rhs[c:c + 12]) for c in col.values()])
    delta = np.zeros_like(dq)
    delta[3] = 1e-5 * np.arange(1, 13)
    d = s.residual(asm.h, q, qd, dq + delta, lam)
    assert d[oracle.RHO_P] == pytest.approx(np.linalg.norm(delta) / np.linalg.norm(hf), rel=1e-6)


def test_post_step_constraints():
    """c_ball is the largest anchor distance |A_a p_a + t_a - A_b p_b - t_b|
    over ball joints (world sides: the stored world point), computed here from
    the state; c_hinge the largest |C| of the hinge rows."""
    asm, s, q, qd = case()
    rng = np.random.default_rng(6)
    qn = q.copy()
    qn[2:6, 9:] += rng.normal(0, 1e-3, (4, 3))
    qn[4, :9] += rng.normal(0, 1e-3, 9)

    def point(b, p):
        if b < 0:
            return p
        A = qn[b, :9].reshape(3, 3).T
        return A @ p + qn[b, 9:]

    cb = max(np.abs(point(asm.ja[k], asm.pa[k]) - point(asm.jb[k], asm.pb[k])).max()
             for k in range(asm.m) if asm.jtype[k] == 0)
    ch = max(np.abs(s.joint_terms(qn, k)[0]).max() for k in range(asm.m) if asm.jtype[k] == 1)
    d = s.residual(asm.h, q, qd, np.zeros_like(q), np.zeros(s.rows), q_new=qn)
    assert d[oracle.CBALL] == pytest.approx(cb, rel=1e-12)
    assert d[oracle.CHINGE] == pytest.approx(ch, rel=1e-12)
    assert cb > 1e-4 and ch > 1e-4
    # without q_new the constraints are evaluated at q + dq
    d2 = s.residual(asm.h, q, qd, qn - q, np.zeros(s.rows))
    assert d2[oracle.CBALL] == pytest.approx(cb, rel=1e-6)


def rodrigues(w):
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th == 0.0:
        return np.eye(3)
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def test_hinge_gradient_along_rigid_motions_away_from_rest():
    """Away from d_m = 0 the hinge gradient's rotation term (Eqs. pcpr,
    r_gradient, A-linearised) is exact along rigid motions: at A = R0 in SO(3)
    a rotation A(e) = exp(e W) R0 moves the polar factor as dR/de = W R0 = dA/de,
    so G times that direction equals the derivative of C.  Checked by central
    differences for both sides' rotations and translations (side b has no
    rotation term: every one of its 12 directions is checked) with d_m != 0;
    the frozen-frame gradient alone fails the same check."""
    asm = mi.chain(3, seed=13, hinge_frac=1.0, sigma=0.0, pin_first=False)
    rng = np.random.default_rng(14)
    for b in range(asm.n):
        R0 = rodrigues(rng.normal(size=3) * 0.5)
        for c in range(3):
            asm.q0[b, 3 * c:3 * c + 3] = R0[:, c]
        asm.q0[b, 9:] += rng.normal(0, 0.03, 3)
    worst = {0: 0.0, 2: 0.0}
    for hg in (0, 2):
        s = oracle.System(asm, hinge_grad=hg)
        q = asm.q0.copy()
        for k in range(asm.m):
            C, Ga, Gb = s.joint_terms(q, k)
            assert np.abs(C).max() > 1e-3    # d_m != 0
            for side, G in ((asm.ja[k], Ga), (asm.jb[k], Gb)):
                A0 = q[side, :9].reshape(3, 3).T
                dirs = []
                for axis in np.eye(3):
                    W = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
                    path = (lambda e, A0=A0, axis=axis: rodrigues(e * axis) @ A0)
                    dirs.append((path, (W @ A0).T.reshape(9), np.zeros(3)))
                for i in range(3):
                    dirs.append((lambda e, A0=A0: A0, np.zeros(9), np.eye(3)[i]))
                if side == asm.jb[k]:
                    for j in range(9):
                        E = np.zeros(9); E[j] = 1.0
                        dirs.append((lambda e, A0=A0, E=E: A0 + e * E.reshape(3, 3).T, E, np.zeros(3)))
                for path, dA, dt in dirs:
                    e = 1e-6
                    qp = q.copy(); qm = q.copy()
                    qp[side, :9] = path(e).T.reshape(9); qp[side, 9:] += e * dt
                    qm[side, :9] = path(-e).T.reshape(9); qm[side, 9:] -= e * dt
                    fd = (s.joint_terms(qp, k)[0] - s.joint_terms(qm, k)[0]) / (2 * e)
                    worst[hg] = max(worst[hg], np.abs(G @ np.concatenate([dA, dt]) - fd).max())
    assert worst[0] < 1e-8
    assert worst[2] > 1e-4
