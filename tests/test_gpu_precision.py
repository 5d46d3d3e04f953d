"""Precision form 1 on chain components: FP32 body solve and dual assembly,
FP64 factor, FP64 KKT residual and correction sweeps until the KKT residual
max(rho_p, rho_d) is at most kkt_tol.

Form 1 must land on the same per-step KKT solution as the plain FP64 path, so
it is held to the same parity bar against the oracle (relative 1e-10 on q and
qdot), and the device-side residual it reports must meet its target.
"""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors
from test_gpu_parity import TOL, teacher_forced

pytestmark = pytest.mark.gpu

F1 = dict(precision=1, kkt_tol=1e-12)


@pytest.mark.parametrize("n", [3, 64, 125, 126, 2049])
def test_form1_chain_sizes(n):
    """Chain lengths around the 62-row tiles of the 64-thread kernels."""
    asm = mi.chain(n, seed=100 + n)
    asm.qd0[1:] = np.random.default_rng(n).normal(0, 0.05, (n - 1, 12))
    say("form 1 chain", n)
    say("worst", teacher_forced(asm, 3, **F1))


def test_form1_chain_variants():
    a = mi.chain(300, seed=101, pin_first=False)
    say("form 1 free chain")
    teacher_forced(a, 2, **F1)
    c = mi.chain(300, seed=102)
    sw = np.arange(0, 299, 2)
    c.ja[sw], c.jb[sw] = c.jb[sw].copy(), c.ja[sw].copy()
    c.pa[sw], c.pb[sw] = c.pb[sw].copy(), c.pa[sw].copy()
    say("form 1 chain with reversed joints")
    teacher_forced(c, 2, **F1)
    d = mi.chain(300, seed=103)
    d.material = 1
    d.poisson = np.full(d.n, 0.3)
    say("form 1 chain, Lame material")
    teacher_forced(d, 2, **F1)


def test_form1_reports_residual_and_sweeps():
    import paper_2603_08079_amd as pk

    asm = mi.chain(5000, seed=104)
    asm.qd0[1:] = np.random.default_rng(104).normal(0, 0.05, (asm.n - 1, 12))
    ctx = pk.Context(asm, **F1)
    s = oracle.System(asm)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for n in range(3):
        ctx.step(asm.h, 1)
        st = ctx.stats()
        q, qd, lam, d = s.step(asm.h, q, qd)
        qg, qdg = ctx.state()
        eq, eqd = state_errors(qg, qdg, q, qd)
        say(n, "sweeps", st["ir_sweeps"], "rho_p", st["rho_p"], "rho_d", st["rho_d"], "err", eq, eqd)
        assert 1 <= st["ir_sweeps"] <= 4
        assert st["kkt"] <= max(F1["kkt_tol"], 2 * d[oracle.KKT])
        assert st["kkt"] == max(st["rho_p"], st["rho_d"])
        assert eq < TOL * (n + 1) and eqd < TOL * (n + 1)


def test_form1_mixed_with_tree():
    """Form 1 covers chain components; a tree in the same context stays FP64."""
    import paper_2603_08079_amd as pk

    parts = [mi.chain(700, seed=105), mi.tree(200, seed=106, origin=(0.0, 25.0, 0.0))]
    asm = mi.concat(parts, h=1e-2, steps=2)
    ctx = pk.Context(asm, **F1)
    assert ctx.stats()["n_chain"] == 1 and ctx.stats()["n_tree"] >= 1
    ref = pk.Context(asm)
    for _ in range(2):
        ctx.step(asm.h, 1)
        ref.step(asm.h, 1)
    q1, qd1 = ctx.state()
    q0, qd0 = ref.state()
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    say("form 1 vs plain", eq, eqd)
    assert eq < TOL and eqd < 1e-9


def test_form1_graph_replay_matches_eager():
    import paper_2603_08079_amd as pk

    asm = mi.chain(3000, seed=107)
    g = pk.Context(asm, use_graph=1, **F1)
    e = pk.Context(asm, use_graph=0, **F1)
    for n in (1, 3, 2):
        g.step(asm.h, n)
        e.step(asm.h, n)
        assert g.stats()["graph_replay"] == 1 and e.stats()["graph_replay"] == 0
        qg, qdg = g.state()
        qe, qde = e.state()
        assert np.array_equal(qg, qe) and np.array_equal(qdg, qde)
        assert g.stats()["ir_sweeps"] == e.stats()["ir_sweeps"]
        assert g.stats()["kkt"] == e.stats()["kkt"]


def test_form1_not_converged_keeps_state():
    """Without correction sweeps the FP32 solve stays far above the target."""
    import paper_2603_08079_amd as pk

    asm = mi.chain(500, seed=108)
    ctx = pk.Context(asm, precision=1, kkt_tol=1e-12, ir_max_sweeps=0)
    q0, qd0 = ctx.state()
    ctx.step(asm.h, 2)  # queued: mabd_multipliers reads the outcome
    with pytest.raises(pk.MabdError) as ei:
        ctx.multipliers()
    assert ei.value.status == pk.ERR_NOT_CONVERGED
    st = ctx.stats()
    say("kkt of the FP32 solve", st["kkt"])
    assert st["ir_sweeps"] == 0 and st["kkt"] > 1e-12
    q1, qd1 = ctx.state()
    assert np.array_equal(q0, q1) and np.array_equal(qd0, qd1)


def test_form1_full_size_chain_one_step():
    """The 1,048,576-body chain in form 1, as the benchmark runs it: one step
    from a moving state against the oracle's block Thomas solve."""
    import paper_2603_08079_amd as pk

    asm = mi.config("chain1m")
    rng = np.random.default_rng(21)
    asm.qd0[1:, 9:] = rng.normal(0, 0.05, (asm.n - 1, 3))
    ctx = pk.Context(asm, precision=1, kkt_tol=1e-12)
    ctx.step(asm.h, 1)
    st = ctx.stats()
    qg, qdg = ctx.state()
    s = oracle.System(asm)
    q1, qd1, lam, d = s.step(asm.h, asm.q0, asm.qd0)
    eq, eqd = state_errors(qg, qdg, q1, qd1)
    say("chain1m form 1: sweeps", st["ir_sweeps"], "kkt", st["kkt"], "err", eq, eqd,
        "oracle kkt", d[oracle.KKT])
    # the same KKT residual as the oracle's direct FP64 solve reaches there
    assert st["kkt"] <= max(1e-12, 2 * d[oracle.KKT])
    assert eq < TOL and eqd < TOL
