"""Path components on the GPU: tree components whose bodies carry at most
two joints each (hinge chains, chains of every joint type, free-floating
chains, chains with world joints at their ends) take the segmented
block-tridiagonal elimination of the dual over their joints (Sec. 5.3).

* parity with the FP64 oracle at 1e-10 (state and multipliers), teacher
  forced, on path lengths around the segment length (16 joints) and its
  multiples;
* segment lengths of 2, 3 and 5 joints (environment, read at create): small
  paths then take several levels of separators;
* the same assemblies through the tree contraction (path_solver = 0): both
  are exact, so states agree to rounding;
* a batch of ragged paths beside trees and ball chains, the path solve on
  a second stream beside the contraction (bitwise the sequential step), the
  form-1 refinement on paths, paths beside a loop-breaker component, several
  Newton iterations, external wrenches, the device KKT residual, and a
  full-size batch against the contraction."""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors, rel_err
from test_gpu_parity import TOL, teacher_forced

pytestmark = pytest.mark.gpu

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None


def moving(asm, seed, sd=0.05):
    asm.qd0[:] = np.random.default_rng(seed).normal(0, sd, asm.qd0.shape)
    asm.qd0[asm.pinned == 1] = 0.0
    return asm


def stats_of(asm, **kw):
    import paper_2603_08079_amd as pk

    ctx = pk.Context(asm, **kw)
    st = ctx.stats()
    ctx.close()
    return st


def run(asm, steps, **kw):
    import paper_2603_08079_amd as pk

    ctx = pk.Context(asm, **kw)
    ctx.step(asm.h, steps)
    q, qd = ctx.state()
    lam = ctx.multipliers()
    st = ctx.stats()
    ctx.close()
    assert st["last_status"] == 0
    return q, qd, lam, st


@pytest.mark.parametrize("n", [2, 3, 16, 17, 18, 33, 256, 500])
def test_hinge_chain_parity(n):
    asm = moving(mi.chain(n, seed=200 + n, hinge_frac=0.5 if n > 3 else 1.0), 200 + n)
    st = stats_of(asm)
    say("hinge chain", n, "paths", st["n_path"], "levels", st["path_levels"])
    assert st["n_path"] == 1 and st["n_chain"] == 0
    say("worst", teacher_forced(asm, 2))


@pytest.mark.parametrize("seg", [2, 3, 5])
def test_short_segments_many_levels(seg, monkeypatch):
    monkeypatch.setenv("MABD_PATH_SEGMENT", str(seg))
    parts = [mi.chain(n, seed=210 + n, hinge_frac=0.5, origin=(0.0, 10.0 * i, 0.0))
             for i, n in enumerate((2, 3, 4, 7, 31, 120))]
    for p in parts:
        p.jtype[-1] = 1  # at least one hinge: not a ball chain
    asm = moving(mi.concat(parts, h=1e-2, steps=2), 216 + seg)
    st = stats_of(asm)
    say("segment", seg, "paths", st["n_path"], "levels", st["path_levels"])
    assert st["n_path"] == len(parts) and st["path_levels"] >= 3
    say("worst", teacher_forced(asm, 2))


def test_every_joint_type_on_a_path():
    asm = mi.mix_joint_types(mi.chain(150, seed=220), seed=221)
    moving(asm, 222)
    st = stats_of(asm)
    say("joint types", np.bincount(asm.jtype, minlength=4), "paths", st["n_path"])
    assert st["n_path"] == 1
    say("worst", teacher_forced(asm, 2))


def test_path_ends():
    """A free-floating path (its ends are bodies), world joints at both ends
    of a hinge chain, and one body held by two world joints."""
    a = moving(mi.chain(60, seed=230, hinge_frac=0.5, pin_first=False), 230)
    b = mi.chain(60, seed=231, hinge_frac=0.5)
    b.jtype = np.append(b.jtype, 1).astype(np.uint8)
    b.ja = np.append(b.ja, 59).astype(np.int32)
    b.jb = np.append(b.jb, -1).astype(np.int32)
    tip = b.q0[59, 9:] + np.array([0.5, 0.0, 0.0])
    b.pa = np.vstack([b.pa, [0.5, 0.0, 0.0]]); b.pb = np.vstack([b.pb, tip])
    b.axis = np.vstack([b.axis, [0.0, 1.0, 0.0]]); b.cp_len = np.append(b.cp_len, 0.1)
    moving(b, 231)
    # a hinge (axis y) at one end and a ball joint at the other: 8 rows on
    # points that are not collinear, which leave the third column of A free;
    # the body starts deforming along it
    c = mi.free_body(dims=(0.4, 0.1, 0.1), k_orth=1e4, t=(0.0, 0.0, 0.0))
    c.jtype = np.array([1, 0], np.uint8); c.ja = np.array([0, -1], np.int32); c.jb = np.array([-1, 0], np.int32)
    c.pa = np.array([[0.2, 0.0, 0.0], [-0.2, 0.0, 0.0]]); c.pb = np.array([[0.2, 0.0, 0.0], [-0.2, 0.0, 0.0]])
    c.axis = np.array([[0.0, 1.0, 0.0], [0.0, 1.0, 0.0]]); c.cp_len = np.array([0.1, 0.1])
    c.qd0[0, 6:9] = [0.1, 0.2, 0.3]
    for name, asm in (("free-floating", a), ("world joints at both ends", b), ("one body, two world joints", c)):
        st = stats_of(asm)
        say(name, "paths", st["n_path"])
        assert st["n_path"] == 1
        say("worst", teacher_forced(asm, 2))


def ragged_batch(seed, count=40, longest=90):
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(count):
        n = int(rng.integers(2, longest))
        if i % 5 == 4:
            parts.append(mi.tree(n + 5, seed=seed + i, window=4, origin=(0.0, 10.0 * i, 0.0)))
        elif i % 7 == 6:
            parts.append(mi.chain(n + 3, seed=seed + i, origin=(0.0, 10.0 * i, 0.0)))  # ball chain
        else:
            parts.append(mi.chain(n, seed=seed + i, hinge_frac=0.5, pin_first=i % 3 != 1,
                                  origin=(0.0, 10.0 * i, 0.0)))
    return moving(mi.concat(parts, h=1e-2, steps=3), seed)


def test_ragged_batch_parity():
    asm = ragged_batch(240)
    st = stats_of(asm)
    say("ragged batch", asm.n, "paths", st["n_path"], "trees", st["n_tree"], "chains", st["n_chain"],
        "levels", st["path_levels"])
    assert st["n_path"] >= 20 and st["n_chain"] >= 1 and st["n_tree"] > st["n_path"]
    say("worst", teacher_forced(asm, 2))


@pytest.mark.parametrize("seg", [None, "3"])
def test_path_solver_matches_contraction(seg, monkeypatch):
    if seg:
        monkeypatch.setenv("MABD_PATH_SEGMENT", seg)
    asm = ragged_batch(250)
    q1, qd1, l1, s1 = run(asm, 3)
    q0, qd0, l0, s0 = run(asm, 3, path_solver=0)
    assert s0["n_path"] == 0 and s1["n_path"] > 0
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    el = rel_err(l1, l0)
    say("path vs contraction: q", eq, "qdot", eqd, "lambda", el)
    # two exact eliminations in different orders, three free-running steps:
    # they differ by about kappa(S) times the rounding unit (measured: q
    # 1.7e-15, qdot 2.1e-11, multipliers 1.2e-10 of the largest); an indexing
    # mistake in either would show at O(1)
    assert eq < 1e-12 and eqd < 1e-10 and el < 1e-9


def test_forked_path_solve_equals_sequential():
    """With trees beside the paths the step's path solve runs on a second
    stream, joined before the back-projection; with kernel groups timed
    (diagnostics bit 1) it runs in sequence.  The two solves touch disjoint
    data, so the states are bitwise equal, eagerly and from a replayed
    graph."""
    asm = ragged_batch(270, count=400, longest=160)  # over 16,384 path joints: forked
    q0, qd0, l0, s0 = run(asm, 4, diagnostics=2)
    q1, qd1, l1, s1 = run(asm, 4)
    q2, qd2, l2, s2 = run(asm, 4, use_graph=0)
    say("graph replay", s1["graph_replay"], "eager", s2["graph_replay"])
    assert s1["graph_replay"] == 1 and s2["graph_replay"] == 0
    for q, qd, lam in ((q1, qd1, l1), (q2, qd2, l2)):
        assert np.array_equal(q, q0) and np.array_equal(qd, qd0) and np.array_equal(lam, l0)


def test_path_form1():
    F1 = dict(precision=1, kkt_tol=1e-12)
    asm = moving(mi.chain(300, seed=260, hinge_frac=0.5), 260)
    say("form 1 on a path")
    say("worst", teacher_forced(asm, 3, tol_v=TOL, **F1))
    q, qd, _, st = run(asm, 3, **F1)
    say("sweeps", st["ir_sweeps"], "kkt", st["kkt"])
    assert st["n_path"] == 1 and st["ir_sweeps"] >= 1
    assert st["kkt"] <= 1e-12 or (st["ir_stalled"] and st["kkt"] <= 1e-11)


def test_full_size_batch_against_contraction():
    """The 4,096-assembly batch: its 2,452 chains with hinges are paths.  One
    step through the path solver against the same step through the tree
    contraction, and the oracle's FP64 KKT residual of the path solver's
    multipliers."""
    asm = mi.config("batch4096")
    say("batch4096", asm.n)
    q1, qd1, l1, s1 = run(asm, 1)
    say("paths", s1["n_path"], "levels", s1["path_levels"])
    q0, qd0, l0, _ = run(asm, 1, path_solver=0)
    eq, eqd = state_errors(q1, qd1, q0, qd0)
    say("path vs contraction: q", eq, "qdot", eqd, "lambda", rel_err(l1, l0))
    assert s1["n_path"] >= 2452  # the chains, and tree components below a pinned root that are paths
    assert eq < 1e-12 and eqd < 1e-9
    s = oracle.System(asm)
    _, _, dv = s.finish(asm.h, asm.q0, asm.qd0, l1)
    say("oracle kkt of the path solver's multipliers", dv[:3])
    assert dv[oracle.KKT] < 1e-10


def test_paths_beside_a_loop_component():
    """A hinge chain (path) and a tree closed by two extra joints (the
    loop-breaker's component) in one context: the loop-breaker's extra tree
    solves run the path solve into their own columns, the step's multipliers
    stay those of the direct solve."""
    from test_gpu_loops import run_against_direct, tree_with_loops

    h = moving(mi.chain(200, seed=280, hinge_frac=0.5, origin=(0.0, 30.0, 0.0)), 280)
    asm = mi.concat([h, tree_with_loops(300, 2, 281)], h=1e-2, steps=2)
    st = stats_of(asm)
    say("paths", st["n_path"], "loops", st["n_loop"])
    assert st["n_path"] >= 1
    say("worst", run_against_direct(asm, 2, expect_loops=1))


def test_path_newton_iterations():
    asm = moving(mi.chain(200, seed=282, hinge_frac=0.5), 282)
    say("worst", teacher_forced(asm, 2, newton_iters=3))


def test_path_wrenches():
    from test_gpu_wrench import compare, wrenches

    asm = moving(mi.mix_joint_types(mi.chain(200, seed=283), seed=284), 283)
    say("worst", compare(asm, wrenches(asm, 285), 2))


def test_path_device_residual():
    """Diagnostics bit 0 on a path: the device's FP64 KKT residual and the
    oracle's verifier on the same GPU step are both at rounding level, and
    the hinges' value after the linearised step agrees closely."""
    from test_gpu_boundary import oracle_check, rounding_level

    asm = moving(mi.chain(400, seed=286, hinge_frac=0.5), 286)
    import paper_2603_08079_amd as pk

    ctx = pk.Context(asm, diagnostics=1)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for n in range(2):
        ctx.step(asm.h, 1)
        st = ctx.stats()
        qg, qdg = ctx.state()
        lam = ctx.multipliers()
        o = oracle_check(asm, q, qd, qg, qdg, lam)
        say(n, "device", {k: st[k] for k in ("rho_p", "rho_d", "kkt", "c_ball", "c_hinge")}, "oracle", o)
        assert st["n_path"] == 1
        assert rounding_level(st["rho_p"], o["rho_p"], 1e-11)
        assert rounding_level(st["rho_d"], o["rho_d"], 1e-10)
        assert o["c_hinge"] > 1e-9 and abs(st["c_hinge"] - o["c_hinge"]) <= 1e-6 * o["c_hinge"]
        q, qd = qg, qdg
    ctx.close()


def test_full_size_hinge_chain_one_step():
    """A 1,048,576-body chain with ball and hinge joints 50/50 (nine levels
    of separators), one step from a moving state in the launch configuration
    the benchmark times, against the oracle's sparse direct solve."""
    asm = moving(mi.config("hchain1m"), 290, sd=0.02)
    import paper_2603_08079_amd as pk

    ctx = pk.Context(asm)
    ctx.step(asm.h, 1)
    st = ctx.stats()
    qg, qdg = ctx.state()
    lam_g = ctx.multipliers()
    ctx.close()
    say("hchain1m: paths", st["n_path"], "levels", st["path_levels"], "graph replay", st["graph_replay"])
    assert st["n_path"] == 1 and st["path_levels"] >= 8 and st["graph_replay"] == 1
    s = oracle.System(asm)
    q1, qd1, lam, d = s.step_sparse(asm.h, asm.q0, asm.qd0)
    eq, eqd = state_errors(qg, qdg, q1, qd1)
    _, _, dv = s.finish(asm.h, asm.q0, asm.qd0, lam_g)
    say("errors", eq, eqd, "oracle kkt", d[:3], "kkt of GPU multipliers", dv[:3])
    assert eq < TOL and eqd < TOL
    assert dv[oracle.KKT] <= max(10 * d[oracle.KKT], 1e-11)
