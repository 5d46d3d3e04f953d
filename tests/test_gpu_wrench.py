"""External wrenches (Eq. module1-wrench-map) on the GPU against the FP64
oracle: every solver path (free bodies, the fused chain path, the tree
contraction, the ball-network PCG), precision form 1, and the step graphs,
which must be re-captured when wrenches are set or removed."""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors

pytestmark = pytest.mark.gpu
TOL = 1e-10
TOL_V_TREE = TOL  # the parity tests' tree bar


def wrenches(asm, seed, scale=1.0):
    """Torques and forces of the order of the bodies' weight times their size."""
    rng = np.random.default_rng(seed)
    m = asm.density * asm.dims.prod(axis=1)
    W = rng.normal(size=(asm.n, 6))
    W[:, :3] *= (scale * 9.8 * m * asm.dims.max(axis=1))[:, None]
    W[:, 3:] *= (scale * 9.8 * m)[:, None]
    return W


def compare(asm, W, steps, tol_v=TOL, **kw):
    """Teacher-forced: both sides start every step from the oracle's state."""
    import paper_2603_08079_amd as pk

    s = oracle.System(asm, wrench=W)
    ctx = pk.Context(asm, **kw)
    ctx.set_wrenches(W)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    worst = (0.0, 0.0)
    for _ in range(steps):
        ctx.set_state(q, qd)
        ctx.step(asm.h, 1)
        qg, qdg = ctx.state()
        if s.classify() == 2 and s.rows > 4000:
            q1, qd1, lam, d = s.step_sparse(asm.h, q, qd)
        else:
            q1, qd1, lam, d = s.step(asm.h, q, qd, solver=oracle.DENSE if s.rows <= 4000 else oracle.AUTO)
        eq, eqd = state_errors(qg, qdg, q1, qd1)
        worst = (max(worst[0], eq), max(worst[1], eqd))
        assert eq < TOL and eqd < tol_v, (eq, eqd)
        q, qd = q1, qd1
    ctx.close()
    return worst


def test_free_bodies_with_wrenches():
    parts = []
    rng = np.random.default_rng(60)
    for i in range(6):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        ang = rng.uniform(0, 3)
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        A = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
        qd = np.zeros(12)
        qd[9:] = rng.normal(size=3)
        parts.append(mi.free_body(dims=tuple(rng.uniform(0.05, 0.4, 3)), A=A, t=(0.0, 2.0 * i, 0.0), qd=qd))
    asm = mi.concat(parts, h=1e-2, steps=3)
    say("free bodies", "worst", compare(asm, wrenches(asm, 61), 3))


def test_chain_with_wrenches():
    asm = mi.chain(300, seed=62)
    say("ball chain 300 (fused chain path)", "worst", compare(asm, wrenches(asm, 63), 3))


def test_tree_with_wrenches():
    asm = mi.tree(400, seed=64)
    say("tree 400 (contraction)", "worst", compare(asm, wrenches(asm, 65), 2, tol_v=TOL_V_TREE))


def test_lattice_with_wrenches():
    asm = mi.lattice(6, seed=66)
    say("lattice 6x6 (PCG)", "worst", compare(asm, wrenches(asm, 67, 0.1), 2, kkt_tol=1e-13))


def test_precision_form_1_with_wrenches():
    """FP32 body solve and assembly, FP64 factor and refinement: the wrench
    enters the FP32 solve and the FP64 residual alike."""
    import paper_2603_08079_amd as pk

    asm = mi.chain(2000, seed=68)
    W = wrenches(asm, 69)
    s = oracle.System(asm, wrench=W)
    ctx = pk.Context(asm, precision=1, kkt_tol=1e-12)
    ctx.set_wrenches(W)
    ctx.step(asm.h, 1)
    qg, qdg = ctx.state()
    q1, qd1, _, _ = s.step(asm.h, asm.q0, asm.qd0)
    eq, eqd = state_errors(qg, qdg, q1, qd1)
    say("form 1 with wrenches", eq, eqd, "sweeps", ctx.stats()["ir_sweeps"])
    assert eq < TOL and eqd < TOL


def test_graphs_follow_wrench_changes():
    """Steps replayed from captured graphs before, while and after wrenches
    are set equal steps of contexts created in each of those states."""
    import paper_2603_08079_amd as pk

    asm = mi.concat([mi.chain(500, seed=70), mi.tree(200, seed=71, origin=(0.0, 20.0, 0.0))], h=1e-2, steps=3)
    W = wrenches(asm, 72)
    ctx = pk.Context(asm)
    ctx.step(asm.h, 2)  # graphs captured without wrenches
    assert ctx.stats()["graph_replay"] == 1
    q, qd = ctx.state()
    ctx.set_wrenches(W)
    ctx.step(asm.h, 2)
    assert ctx.stats()["graph_replay"] == 1
    qa, qda = ctx.state()
    ref = pk.Context(asm, use_graph=0)
    ref.set_state(q, qd)
    ref.set_wrenches(W)
    ref.step(asm.h, 2)
    qr, qdr = ref.state()
    assert np.array_equal(qa, qr) and np.array_equal(qda, qdr)
    ctx.set_wrenches(None)
    ref.set_wrenches(None)
    ctx.step(asm.h, 1)
    ref.step(asm.h, 1)
    qa, qda = ctx.state()
    qr, qdr = ref.state()
    assert np.array_equal(qa, qr) and np.array_equal(qda, qdr)
    # and the wrench did act: a context that never had one differs
    plain = pk.Context(asm, use_graph=0)
    plain.set_state(q, qd)
    plain.step(asm.h, 3)
    assert not np.array_equal(plain.state()[0], qa)


def test_wrench_validation():
    import paper_2603_08079_amd as pk

    asm = mi.chain(20, seed=73)
    ctx = pk.Context(asm)
    W = np.zeros((asm.n, 6))
    W[3, 2] = np.nan
    with pytest.raises(pk.MabdError) as ei:
        ctx.set_wrenches(W)
    assert ei.value.status == pk.ERR_INVALID_ARG
