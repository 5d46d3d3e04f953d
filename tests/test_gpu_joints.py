"""Universal (Eq. universal) and prismatic (Eq. prismatic) joints on the GPU
against the oracle, next to balls and hinges: trees and chains through the
tree contraction (cliques with 3-, 4- and 5-row joints), world-tied joints
(world-owned frames), a network through the general PCG, and the post-step
joint values of the device diagnostics.  Same bar as every other assembly:
the state to 1e-10 of the oracle's, per step."""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors
from test_gpu_parity import TOL, teacher_forced
from test_oracle_joint_pins import mixed_assemblies

pytestmark = pytest.mark.gpu

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None


def test_mixed_joint_tree():
    t = mi.mix_joint_types(mi.tree(400, seed=91), seed=92)
    t.qd0[1:] = np.random.default_rng(93).normal(0, 0.05, (t.n - 1, 12))
    say("tree of 400 with ball, hinge, universal and prismatic joints", np.bincount(t.jtype))
    say("worst", teacher_forced(t, 3, tol_v=TOL))


def test_universal_and_prismatic_chains():
    for probs, name in (((0, 0, 1, 0), "universal"), ((0, 0, 0, 1), "prismatic"),
                        ((0.3, 0.2, 0.25, 0.25), "mixed")):
        c = mi.mix_joint_types(mi.chain(600, seed=94), seed=95, probs=probs)
        c.qd0[1:] = np.random.default_rng(96).normal(0, 0.05, (c.n - 1, 12))
        say(name, "chain of 600")
        say("worst", teacher_forced(c, 2, tol_v=TOL))


@pytest.mark.parametrize("name,asm", mixed_assemblies(), ids=lambda x: x if isinstance(x, str) else "")
def test_world_tied_mixed_joints(name, asm):
    say(name)
    say("worst", teacher_forced(asm, 3, tol_v=TOL))


def test_mixed_joint_trees_in_one_context():
    parts = [mi.mix_joint_types(mi.tree(n, seed=100 + n, window=w, origin=(0.0, 20.0 * i, 0.0)),
                                seed=200 + n)
             for i, (n, w) in enumerate(((900, 64), (60, 2), (300, 8), (7, 1)))]
    asm = mi.concat(parts, h=1e-2, steps=2)
    asm.qd0[:] = np.random.default_rng(97).normal(0, 0.05, asm.qd0.shape)
    asm.qd0[asm.pinned == 1] = 0.0
    say("mixed-joint trees in one context", asm.n)
    say("worst", teacher_forced(asm, 2, tol_v=TOL))


def test_mixed_joint_network_pcg():
    """A lattice whose joints are of all four types: loops, solved by the
    general PCG; compared with the oracle's sparse direct solve."""
    import paper_2603_08079_amd as pk

    asm = mi.mix_joint_types(mi.lattice(6, seed=98), seed=99)
    s = oracle.System(asm)
    ctx = pk.Context(asm, kkt_tol=1e-12)
    assert ctx.stats()["n_graph"] == 1
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for n in range(2):
        ctx.set_state(q, qd)
        ctx.step(asm.h, 1)
        qg, qdg = ctx.state()
        lam_g = ctx.multipliers()
        q1, qd1, lam, d = s.step_sparse(asm.h, q, qd)
        _, _, dv = s.finish(asm.h, q, qd, lam_g)
        eq, eqd = state_errors(qg, qdg, q1, qd1)
        say(n, "pcg iters", ctx.stats()["pcg_iters"], "errors", eq, eqd, "oracle kkt of GPU lam", dv[:3])
        assert dv[oracle.RHO_D] <= 2e-12
        assert eq < TOL and eqd < 1e-5
        q, qd = q1, qd1


def test_joint_values_after_a_step():
    """The device's post-step joint values of the rotated-frame joints (their
    nonlinear drift) agree with the oracle's."""
    import paper_2603_08079_amd as pk

    t = mi.mix_joint_types(mi.tree(300, seed=101), seed=102, probs=(0.0, 0.0, 0.5, 0.5))
    t.qd0[1:] = np.random.default_rng(103).normal(0, 0.05, (t.n - 1, 12))
    ctx = pk.Context(t, diagnostics=1)
    ctx.step(t.h, 1)
    st = ctx.stats()
    qg, qdg = ctx.state()
    lam = ctx.multipliers()
    d = oracle.System(t).residual(t.h, t.q0, t.qd0, qdg * t.h, lam, q_new=qg)
    say("c_other device", st["c_hinge"], "oracle", d[oracle.CHINGE], "kkt", st["kkt"], d[oracle.KKT])
    assert d[oracle.CHINGE] > 1e-9
    assert abs(st["c_hinge"] - d[oracle.CHINGE]) <= 1e-6 * d[oracle.CHINGE]
    assert st["kkt"] < 1e-10 and d[oracle.KKT] < 1e-10


def test_vertical_slider_on_the_gpu():
    """The prismatic slider of the oracle pins: closed-form free fall."""
    import paper_2603_08079_amd as pk

    body = mi.free_body(dims=(0.2, 0.3, 0.4), t=(1.0, 2.0, 3.0))
    body.jtype = np.array([mi.PRISMATIC], np.uint8)
    body.ja = np.array([-1], np.int32); body.jb = np.array([0], np.int32)
    body.pa = np.array([[1.0, 2.0, 3.2]]); body.pb = np.array([[0.0, 0.0, 0.2]])
    body.axis = np.array([[0.0, 0.0, 1.0]]); body.axis2 = np.array([[1.0, 0.0, 0.0]])
    body.cp_len = np.array([0.1])
    ctx = pk.Context(body)
    ctx.step(body.h, 30)
    q, qd = ctx.state()
    z = 3.0 - 0.5 * 30 * 31 * body.h ** 2 * 9.8
    say("slider z", q[0, 11], "closed form", z)
    assert abs(q[0, 11] - z) <= 1e-12 * 3.0
    assert np.abs(q[0, 9:11] - [1.0, 2.0]).max() <= 1e-13
