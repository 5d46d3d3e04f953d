"""Pins of the reference network of the learned warm start (CPU).

The network is not part of the paper, so it is pinned by properties that any
correct implementation of its definition has: the energy loss equals the
S-norm error identity of the dual quadratic, the message passing is
equivariant under a renumbering of joints and bodies, and a hand-computed
two-joint case."""
import numpy as np

import mabd_inputs as mi
import oracle
from oracle import gnn_ref as G


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, G.NPARAM)


def _net(asm, lam_prev=None):
    s = oracle.System(asm)
    S, r = s.dual(asm.h, asm.q0, asm.qd0)
    return G.Network(asm, S, r, lam_prev), S, r


def test_energy_identity():
    """The loss is the decrease of the dual energy E(l) = 1/2 l^T S l - r^T l
    from the base start, and E(l) - E(l*) = 1/2 |l - l*|_S^2 with
    l* = S^{-1} r: checked against the plain energy, with and without a base."""
    asm = mi.lattice(5, seed=1)
    for base in (None, np.random.default_rng(8).normal(0.0, 5.0, 3 * asm.m)):
        net, S, r = _net(asm, base)
        p = _params(2)
        lam = net.forward(p).ravel()
        Sd = S.toarray()
        E = lambda l: 0.5 * l @ Sd @ l - r @ l
        lb = np.zeros_like(lam) if base is None else base
        assert abs(net.loss(p) * net.eref - (E(lam) - E(lb))) <= 1e-9 * abs(E(lb) - E(lam)) + 1e-12 * abs(E(lb))
        ls = np.linalg.solve(Sd, r)
        assert abs((E(lam) - E(ls)) - 0.5 * (lam - ls) @ Sd @ (lam - ls)) <= 1e-9 * abs(E(ls))


def test_permutation_equivariance():
    asm = mi.lattice(5, seed=3)
    lam_prev = np.random.default_rng(4).normal(size=3 * asm.m)
    net, _, _ = _net(asm, lam_prev)
    p = _params(5)
    y = net.forward(p)
    perm = np.random.default_rng(6).permutation(asm.m)
    b = asm.copy()
    for f in ("jtype", "ja", "jb", "pa", "pb", "axis", "cp_len"):
        setattr(b, f, getattr(b, f)[perm])
    netp, _, _ = _net(b, lam_prev.reshape(-1, 3)[perm].ravel())
    yp = netp.forward(p)
    assert np.allclose(yp, y[perm], rtol=1e-10, atol=1e-12 * np.abs(y).max())


def test_two_joint_message_by_hand():
    """Chain of 3 bodies, body 0 pinned: joint 0 (world, body 1), joint 1
    (body 1, body 2); deg(1) = 2, deg(2) = 1.  Weights chosen so that h0 =
    deg_b (4 x feature 7), layer 1 copies the neighbour channel, layers 2-3
    and the decoder copy channel 0: the output is the normalised neighbour sum
    n_k = (m_a + m_b) / (deg_a + deg_b) with m_1 = 2 + 1, m_2 = 1, i.e.
    n_0 = 3 / 2 and n_1 = (3 + 1) / 3.  Two more channels check the
    rectifiers: channel 1 of the last layer has bias -1 and feeds output 1;
    channel 2 of the encoder has bias -1 and reaches output 2 through a -1
    weight in layer 1 and unit weights after it.  Both outputs are 0 only if
    every layer clips its negative values."""
    asm = mi.chain(3, seed=7)
    net, _, _ = _net(asm)
    assert list(net.ja) == [-1, 1] and list(net.jb) == [1, 2]
    assert np.allclose(net.x[:, 6:11], [[0.0, 0.5, 1.0, 0.0, 0.0], [0.5, 0.25, 0.0, 0.0, 0.0]])
    p = np.zeros(G.NPARAM)
    p[G.P_WE + 7 * G.W + 0] = 4.0
    p[G.P_L0 + 64 * G.W + 0] = 1.0
    for l in (1, 2):
        p[G.P_L0 + l * G.P_LS + 0] = 1.0
    p[G.P_WD + 0] = 1.0
    p[G.P_L0 + 2 * G.P_LS + 2 * G.W * G.W + 1] = -1.0  # last layer, bias of channel 1
    p[G.P_WD + 1 * 3 + 1] = 1.0
    p[G.P_CE + 2] = -1.0                                 # encoder, bias of channel 2
    p[G.P_L0 + 0 * G.P_LS + 2 * G.W + 2] = -1.0          # layer 1: channel 2 <- -channel 2
    for l in (1, 2):
        p[G.P_L0 + l * G.P_LS + 2 * G.W + 2] = 1.0
    p[G.P_WD + 2 * 3 + 2] = 1.0
    y = net.forward(p) / net.s
    assert np.allclose(y[:, 0], [1.5, 4.0 / 3.0], rtol=1e-14)
    assert np.all(y[:, 1:] == 0.0)
