"""Degenerate assemblies through the C ABI on the GPU: nothing to solve,
nothing dynamic, a single dynamic body on a pinned one, a body held by two
world joints, and all of these mixed into one context with ordinary
components.  Where something moves, the oracle decides."""
import dataclasses

import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors

pytestmark = pytest.mark.gpu
TOL = 1e-10


def empty_assembly():
    z3, z12 = np.zeros((0, 3)), np.zeros((0, 12))
    return mi.Assembly(name="empty", dims=z3, density=np.zeros(0), k_orth=np.zeros(0),
                       pinned=np.zeros(0, np.uint8), q0=z12, qd0=z12, jtype=np.zeros(0, np.uint8),
                       ja=np.zeros(0, np.int32), jb=np.zeros(0, np.int32), pa=z3, pb=z3, axis=z3,
                       cp_len=np.zeros(0))


def check_against_oracle(asm, steps=2, **kw):
    import paper_2603_08079_amd as pk

    ctx = pk.Context(asm, **kw)
    s = oracle.System(asm)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for _ in range(steps):
        ctx.set_state(q, qd)
        ctx.step(asm.h, 1)
        qg, qdg = ctx.state()
        q1, qd1, _, _ = s.step(asm.h, q, qd, solver=oracle.DENSE)
        eq, _ = state_errors(qg, qdg, q1, qd1)
        # velocities against the larger of the outgoing and incoming scales and
        # g h (what gravity alone adds in a step): a step the joints bring to
        # rest leaves only rounding on both sides
        vs = max(float(np.abs(qd1).max(initial=0.0)), float(np.abs(qd).max(initial=0.0)), 9.8 * asm.h)
        eqd = float(np.abs(qdg - qd1).max(initial=0.0)) / vs
        assert eq < TOL and eqd < TOL, (eq, eqd)
        q, qd = q1, qd1
    return ctx


def test_empty_assembly():
    import paper_2603_08079_amd as pk

    asm = empty_assembly()
    ctx = pk.Context(asm)
    ctx.step(1e-2, 3)
    q, qd = ctx.state()
    st = ctx.stats()
    say("empty:", q.shape, st["n_dyn"], st["n_chain"], st["n_tree"], st["n_graph"])
    assert q.shape == (0, 12) and st["n_dyn"] == 0 and st["steps_done"] == 3


def test_all_pinned_bodies_stay():
    import paper_2603_08079_amd as pk

    asm = mi.concat([mi.free_body(t=(float(i), 0.0, 0.0)) for i in range(4)], h=1e-2, steps=2)
    asm = dataclasses.replace(asm, pinned=np.ones(4, np.uint8))
    ctx = pk.Context(asm)
    ctx.step(asm.h, 5)
    q, qd = ctx.state()
    assert np.array_equal(q, asm.q0) and not np.any(qd)


def test_single_body_on_pinned_body():
    asm = mi.chain(2, seed=80)
    asm.qd0[1] = np.random.default_rng(80).normal(0, 0.05, 12)
    ctx = check_against_oracle(asm, 3)
    say("chain of 2: classes", ctx.stats()["n_chain"], ctx.stats()["n_tree"], ctx.stats()["n_graph"])


def test_body_with_two_world_joints():
    """Two ball joints from one body to fixed world points (6 rows on one
    body): a one-body component with two one-sided joints."""
    body = mi.free_body(dims=(0.4, 0.1, 0.1), t=(0.0, 0.0, 1.0))
    asm = dataclasses.replace(
        body, jtype=np.zeros(2, np.uint8), ja=np.array([0, 0], np.int32), jb=np.array([-1, -1], np.int32),
        pa=np.array([[0.2, 0.0, 0.0], [-0.2, 0.0, 0.0]]), pb=np.array([[0.2, 0.0, 1.0], [-0.2, 0.0, 1.0]]),
        axis=np.zeros((2, 3)), cp_len=np.zeros(2))
    asm.qd0[0, 9:] = [0.0, 0.3, 0.0]
    check_against_oracle(asm, 3)


def test_degenerate_components_mixed_with_ordinary_ones():
    parts = [mi.chain(2, seed=81, origin=(0.0, 0.0, 0.0)),
             mi.free_body(t=(0.0, 5.0, 0.0)),
             mi.chain(40, seed=82, origin=(0.0, 10.0, 0.0)),
             mi.tree(30, seed=83, origin=(0.0, 20.0, 0.0)),
             mi.lattice(3, seed=84)]
    parts[-1] = dataclasses.replace(parts[-1], q0=parts[-1].q0.copy())
    parts[-1].q0[:, 9:] += [0.0, 30.0, 0.0]
    asm = mi.concat(parts, h=1e-2, steps=2)
    asm.qd0[:, 9:] += np.random.default_rng(85).normal(0, 0.05, (asm.n, 3)) * (asm.pinned == 0)[:, None]
    check_against_oracle(asm, 2, kkt_tol=1e-13)  # the lattice takes the PCG path
