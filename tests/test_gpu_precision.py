"""Precision form 1: FP32 body solve and dual assembly, FP64 factor, FP64 KKT
residual and correction sweeps until the KKT residual max(rho_p, rho_d) is at
most kkt_tol.  Chain components run it on the fused chain path (device-side
sweep control); tree components (contexts without loop or network
components) in the tree contraction, the force and local solve and the
clique matrices in FP32, the sweeps under host control.

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
    """Form 1 on a chain and a tree in one context lands on the plain FP64
    solution."""
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


# ------------------------------------------------------------ tree components
def test_form1_tree_parity():
    """Trees (ball and hinge joints), a hinge chain (tree path) and a tree of
    all four joint types, every step against the oracle at the FP64 bar."""
    t = mi.tree(400, seed=111)
    t.qd0[1:] = np.random.default_rng(111).normal(0, 0.05, (t.n - 1, 12))
    say("form 1 tree of 400")
    say("worst", teacher_forced(t, 3, tol_v=TOL, **F1))
    c = mi.chain(500, seed=112, hinge_frac=0.5)
    c.qd0[1:] = np.random.default_rng(112).normal(0, 0.05, (c.n - 1, 12))
    say("form 1 hinge chain of 500")
    say("worst", teacher_forced(c, 3, tol_v=TOL, **F1))
    m = mi.mix_joint_types(mi.tree(300, seed=113), seed=114)
    m.qd0[1:] = np.random.default_rng(113).normal(0, 0.05, (m.n - 1, 12))
    say("form 1 mixed-joint tree of 300")
    say("worst", teacher_forced(m, 3, tol_v=TOL, **F1))


def test_form1_tree_world_joints():
    from test_oracle_joint_pins import mixed_assemblies

    for name, asm in mixed_assemblies():
        say("form 1", name)
        say("worst", teacher_forced(asm, 2, tol_v=TOL, **F1))


def test_form1_tree_reports_residual_and_sweeps():
    import paper_2603_08079_amd as pk

    t = mi.tree(3000, seed=115)
    t.qd0[1:] = np.random.default_rng(115).normal(0, 0.05, (t.n - 1, 12))
    ctx = pk.Context(t, **F1)
    plain = pk.Context(t, diagnostics=1)
    for n in range(3):
        ctx.step(t.h, 1)
        plain.step(t.h, 1)
        st, sp = ctx.stats(), plain.stats()
        say(n, "sweeps", st["ir_sweeps"], "stalled", st["ir_stalled"], "kkt", st["kkt"],
            "plain FP64 kkt", sp["kkt"])
        assert 1 <= st["ir_sweeps"] <= 4 and st["last_status"] == 0
        assert st["kkt"] == max(st["rho_p"], st["rho_d"])
        assert st["kkt"] <= F1["kkt_tol"] or (st["ir_stalled"] and st["kkt"] <= 10 * F1["kkt_tol"])
    q1, qd1 = ctx.state()
    q0, qd0 = plain.state()
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    say("form 1 vs plain after 3 steps", eq, eqd)
    assert eq < TOL and eqd < TOL


def test_form1_tree_not_converged_keeps_state():
    """Without correction sweeps the FP32 tree solve stays above the target;
    the step waits for its checks, so mabd_step itself reports it."""
    import paper_2603_08079_amd as pk

    t = mi.tree(500, seed=116)
    ctx = pk.Context(t, precision=1, kkt_tol=1e-12, ir_max_sweeps=0)
    q0, qd0 = ctx.state()
    with pytest.raises(pk.MabdError) as ei:
        ctx.step(t.h, 2)
    assert ei.value.status == pk.ERR_NOT_CONVERGED
    st = ctx.stats()
    say("kkt of the FP32 tree solve", st["kkt"])
    assert st["ir_sweeps"] == 0 and st["kkt"] > 1e-12 and st["steps_done"] == 0
    q1, qd1 = ctx.state()
    assert np.array_equal(q0, q1) and np.array_equal(qd0, qd1)


def test_form1_batch_of_chains_and_trees():
    """A small batch: ball chains in the fused form 1, hinge chains and trees
    in the tree form 1, against the plain FP64 solve of the same context
    shape."""
    import paper_2603_08079_amd as pk

    asm = mi.concat([mi.batch(24, seed=117, hi=600), mi.chain(800, seed=119, origin=(0.0, -30.0, 0.0))],
                    h=1e-2, steps=2)
    asm.qd0[:] = np.random.default_rng(117).normal(0, 0.05, asm.qd0.shape)
    asm.qd0[asm.pinned == 1] = 0.0
    f1 = pk.Context(asm, **F1)
    p0 = pk.Context(asm)
    st0 = f1.stats()
    say("batch of 24:", asm.n, "bodies, chains", st0["n_chain"], "trees", st0["n_tree"])
    assert st0["n_chain"] >= 1 and st0["n_tree"] >= 1
    for _ in range(2):
        f1.step(asm.h, 1)
        p0.step(asm.h, 1)
        st = f1.stats()
        assert st["last_status"] == 0 and st["ir_sweeps"] >= 1
    q1, qd1 = f1.state()
    q0, qd0 = p0.state()
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    say("form 1 vs plain", eq, eqd, "kkt", f1.stats()["kkt"])
    assert eq < TOL and eqd < TOL


def test_form1_with_loops_stays_fp64():
    """A context with a loop component keeps its generic components FP64 (no
    sweeps are reported for them)."""
    import paper_2603_08079_amd as pk
    from test_gpu_loops import ring

    asm = ring(64, seed=118)
    f1 = pk.Context(asm, **F1)
    p0 = pk.Context(asm)
    assert f1.stats()["n_loop"] == 1
    f1.step(asm.h, 1)
    p0.step(asm.h, 1)
    assert f1.stats()["ir_sweeps"] == 0
    q1, qd1 = f1.state()
    q0, qd0 = p0.state()
    assert np.array_equal(q1, q0) and np.array_equal(qd1, qd0)


def test_form1_full_size_tree_one_step():
    """The 262,144-body tree in form 1 against the plain FP64 GPU solve (both
    at the FP64 floor), as the benchmark runs it."""
    import paper_2603_08079_amd as pk

    asm = mi.config("tree256k")
    f1 = pk.Context(asm, precision=1, kkt_tol=1e-12)
    p0 = pk.Context(asm, diagnostics=1)
    f1.step(asm.h, 1)
    p0.step(asm.h, 1)
    st, sp = f1.stats(), p0.stats()
    q1, qd1 = f1.state()
    q0, qd0 = p0.state()
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    say("tree256k form 1: sweeps", st["ir_sweeps"], "kkt", st["kkt"], "plain kkt", sp["kkt"], "err", eq, eqd)
    assert st["kkt"] <= 1e-12 and eq < TOL and eqd < TOL


def test_form1_tree_stall_far_above_target_is_not_converged():
    """An unreachable target: the tree refinement stalls at the FP64 floor
    (or runs out of sweeps) far above it and reports NOT_CONVERGED."""
    import paper_2603_08079_amd as pk

    t = mi.tree(800, seed=120)
    t.qd0[1:] = np.random.default_rng(120).normal(0, 0.05, (t.n - 1, 12))
    ctx = pk.Context(t, precision=1, kkt_tol=1e-17, ir_max_sweeps=6)
    q0, qd0 = ctx.state()
    with pytest.raises(pk.MabdError) as ei:
        ctx.step(t.h, 1)
    assert ei.value.status == pk.ERR_NOT_CONVERGED
    st = ctx.stats()
    say("stalled at", st["kkt"], "after", st["ir_sweeps"], "sweeps")
    assert st["kkt"] > 1e-16 and st["ir_sweeps"] >= 1 and st["ir_stalled"] == 0
    q1, qd1 = ctx.state()
    assert np.array_equal(q0, q1) and np.array_equal(qd0, qd1)


def test_form1_full_size_batch_one_step():
    """The 4,096-assembly batch (2.95M bodies) in form 1, one step from a
    moving state, against the plain FP64 GPU solve of the same step (both
    at the FP64 floor)."""
    import paper_2603_08079_amd as pk

    asm = mi.config("batch4096")
    asm.qd0[:, 9:] = np.random.default_rng(22).normal(0, 0.05, (asm.n, 3))
    asm.qd0[asm.pinned == 1] = 0.0
    f1 = pk.Context(asm, precision=1, kkt_tol=1e-12)
    p0 = pk.Context(asm, diagnostics=1)
    f1.step(asm.h, 1)
    p0.step(asm.h, 1)
    st, sp = f1.stats(), p0.stats()
    q1, qd1 = f1.state()
    q0, qd0 = p0.state()
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    say("batch4096 form 1: sweeps", st["ir_sweeps"], "kkt", st["kkt"], "plain kkt", sp["kkt"], "err", eq, eqd)
    assert st["last_status"] == 0 and st["kkt"] <= 1e-12
    assert eq < TOL and eqd < TOL
