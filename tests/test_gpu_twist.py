"""Twist and joint-wrench diagnostics on the GPU against the oracle's maps
(Eq. module1-G-twist; E(A)^T of Eq. module2-E applied to the joint forces of
the last step), on chains (fused chain path), trees with hinges and world
joints (tree contraction) and a network (PCG), for the GPU's own state and
multipliers."""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say
from test_gpu_boundary import mixed_tree

pytestmark = pytest.mark.gpu

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None


def cases():
    c = mi.chain(2000, seed=71)
    c.qd0[1:] = np.random.default_rng(71).normal(0, 0.05, (c.n - 1, 12))
    yield "chain", c, {}
    yield "tree", mixed_tree(), {}
    yield "lattice", mi.lattice(10, seed=72), dict(kkt_tol=1e-12)


@pytest.mark.parametrize("name,asm,kw", list(cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_twists_and_joint_wrenches(name, asm, kw):
    import paper_2603_08079_amd as pk

    s = oracle.System(asm)
    ctx = pk.Context(asm, **kw)
    for n in range(2):
        q0, qd0 = ctx.state()
        ctx.step(asm.h, 1)
        q1, qd1 = ctx.state()
        lam = ctx.multipliers()
        V = ctx.twists()
        W = ctx.joint_wrenches()
        Vo = s.twists(q1, qd1)
        Wo = s.joint_wrenches(q0, lam)
        ev = np.abs(V - Vo).max() / max(np.abs(Vo).max(), 1e-300)
        ew = np.abs(W - Wo).max() / max(np.abs(Wo).max(), 1e-300)
        say(name, n, "twist", ev, "wrench", ew, "max |W|", np.abs(Wo).max())
        assert ev < 1e-12 and ew < 1e-12
        assert np.all(V[asm.pinned == 1] == 0) and np.all(W[asm.pinned == 1] == 0)


def test_joint_wrench_needs_a_completed_step():
    import paper_2603_08079_amd as pk

    asm = mi.chain(50, seed=73)
    ctx = pk.Context(asm)
    with pytest.raises(pk.MabdError):
        ctx.joint_wrenches()
    ctx.step(asm.h, 1)
    ctx.joint_wrenches()
