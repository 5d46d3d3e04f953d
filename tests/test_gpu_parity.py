"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: the GPU state matches the oracle's state to
relative 1e-10 per step in FP64.  Positions are compared relative to the
largest coordinate, velocities relative to the largest velocity (a stricter
check of the increment itself).  Multipliers are compared relative to their
largest entry.
"""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-10

try:  # import torch at collection time: its first import on a fresh box is slow
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None


def ctx_of(asm, **kw):
    import paper_2603_08079_amd as pk

    return pk.Context(asm, **kw)


def reference_step(s, asm, q, qd, solver):
    """Oracle step.  Trees use the direct dual solve (dense Cholesky, or SuperLU
    when large): the primal condensation accumulates rounding with depth
    (~1e-11 relative on 300 bodies against brute-force KKT LU), the dual solve
    stays at ~5e-12."""
    if solver == oracle.AUTO and s.classify() == 2:
        if s.rows <= 4000:
            return s.step(asm.h, q, qd, solver=oracle.DENSE)
        if s.s.newton_iters == 1:
            return s.step_sparse(asm.h, q, qd)
    return s.step(asm.h, q, qd, solver=solver)


# Trees are held to the same bar as every other assembly.  The oracle's exact
# FP64 solvers (dense Cholesky and SuperLU of the dual, primal leaf-to-root
# condensation, LU of the full KKT matrix) agree among themselves on tree
# velocities to 6e-12 of the largest velocity on the tree test cases, and the
# GPU's tree contraction to 5e-12; in addition, the oracle's FP64 KKT residual
# of the GPU multipliers must be as small as that of its own solution.
TOL_V_TREE = TOL


def teacher_forced(asm, steps, solver=oracle.AUTO, tol=TOL, tol_v=None, **kw):
    """Both sides start every step from the oracle's state."""
    s = oracle.System(asm, **{k: v for k, v in kw.items() if k in ("material", "hinge_grad", "newton_iters")})
    ctx = ctx_of(asm, **kw)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    worst = (0.0, 0.0, 0.0)
    for n in range(steps):
        ctx.set_state(q, qd)
        ctx.step(asm.h, 1)
        qg, qdg = ctx.state()
        lam_g = ctx.multipliers()
        q1, qd1, lam, d = reference_step(s, asm, q, qd, solver)
        eq, eqd = state_errors(qg, qdg, q1, qd1)
        # multipliers are forces (N): floor the scale at 1e-6 of the total weight,
        # since a freely falling assembly has lambda ~ 0 up to rounding
        wscale = 1e-6 * float((asm.density * asm.dims.prod(axis=1)).sum()) * 9.8
        el = rel_err(lam_g, lam, wscale) if asm.m else 0.0
        worst = tuple(max(a, b) for a, b in zip(worst, (eq, eqd, el)))
        tv = tol if tol_v is None else tol_v
        if tol_v is not None and asm.m:
            _, _, dv = s.finish(asm.h, q, qd, lam_g) if s.s.newton_iters == 1 else (0, 0, d)
            say("  kkt gpu", dv[:3], "oracle", d[:3])
            assert dv[oracle.KKT] <= max(10 * d[oracle.KKT], 1e-11)
        assert eq < tol and eqd < tv, (n, eq, eqd)
        assert el < tol, (n, el)
        q, qd = q1, qd1
    ctx.close()
    return worst


def test_free_spinning_body():
    qd = np.zeros(12)
    om = np.array([1.0, 8.0, 2.0])
    for c in range(3):
        qd[3 * c:3 * c + 3] = np.cross(om, np.eye(3)[:, c])
    qd[9:] = [1.0, 0.0, 0.5]
    b = mi.free_body(dims=(0.3, 0.2, 0.1), k_orth=1e7, qd=qd)
    say("free body", b.n)
    say("worst", teacher_forced(b, 20))


def test_chain64_config_trajectory():
    """The 64-body chain configuration over its 200 steps, free running on
    both sides, plus the exact ball-joint residual of every GPU step."""
    asm = mi.config("chain64")
    say("chain64 trajectory", asm.n, asm.m)
    ctx = ctx_of(asm)
    st = ctx.stats()
    assert st["n_chain"] == 1 and st["n_tree"] == 0
    s = oracle.System(asm)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for n in range(asm.steps):
        ctx.step(asm.h, 1)
        q, qd, lam, d = s.step(asm.h, q, qd)
        if n % 20 == 19 or n < 3:
            qg, qdg = ctx.state()
            eq, eqd = state_errors(qg, qdg, q, qd)
            say(n, eq, eqd)
            # free running: rounding differences may grow with the step count
            assert eq < TOL * (n + 1) and eqd < TOL * (n + 1), (n, eq, eqd)
    qg, _ = ctx.state()
    chk = oracle.System(asm)
    cmax = max(np.abs(chk.joint_terms(qg, k)[0]).max() for k in range(asm.m))
    assert cmax < 1e-13 * max(1.0, np.abs(qg[:, 9:]).max())


def test_chain64_teacher_forced():
    asm = mi.config("chain64")
    asm.qd0[1:] = np.random.default_rng(3).normal(0, 0.1, (63, 12))
    say("chain64 teacher forced")
    say("worst", teacher_forced(asm, 10))


@pytest.mark.parametrize("n", [3, 4, 5, 129, 255, 256, 257, 258, 300, 509, 510, 511, 777, 2049])
def test_chain_tile_edges(n):
    """Chains whose row count lands on, below and above tile boundaries."""
    asm = mi.chain(n, seed=n)
    asm.qd0[1:] = np.random.default_rng(n).normal(0, 0.05, (n - 1, 12))
    say("chain", n)
    say("worst", teacher_forced(asm, 2))


@pytest.mark.parametrize("tt", ["64p", "64"])
def test_chain_tails_in_one_context(tt, monkeypatch):
    """Many chains in one context whose last tiles take every row count from
    1 to 62, so that groups of four packed tiles mix chains, full and ragged
    tiles, and the last group is partial."""
    monkeypatch.setenv("MABD_CHAIN_TILE_THREADS", tt)
    parts = [mi.chain(n, seed=1000 + n) for n in range(3, 130)]
    asm = mi.concat(parts, name="tails")
    asm.qd0 = asm.qd0 + np.random.default_rng(41).normal(0, 0.05, asm.qd0.shape) * (asm.pinned == 0)[:, None]
    say("chain tails", tt, "bodies", asm.n)
    say("worst", teacher_forced(asm, 2))


@pytest.mark.parametrize("tt", ["64p", "64", "256"])
def test_chain_top_system_in_global_memory(tt, monkeypatch):
    """MABD_CHAIN_TOP_GLOBAL=1 sends every chain's top system (the rows that
    bound the groups of interface rows) through chain_global_kernel, the path
    that chains of more than ~3.9M rows take; several chains of different
    group counts in one context, two steps against the oracle."""
    monkeypatch.setenv("MABD_CHAIN_TOP_GLOBAL", "1")
    monkeypatch.setenv("MABD_CHAIN_TILE_THREADS", tt)
    parts = [mi.chain(n, seed=n) for n in (40, 20_000, 70_000, 160_000)]
    asm = mi.concat(parts, name="top_global")
    asm.qd0 = asm.qd0 + np.random.default_rng(43).normal(0, 0.05, asm.qd0.shape) * (asm.pinned == 0)[:, None]
    say("top system in global memory", tt, "bodies", asm.n)
    say("worst", teacher_forced(asm, 2))


def test_chain_variants():
    """No pinned body (free chain), a world joint at the far end, and joints
    listed with reversed sides (flags of the row ends)."""
    a = mi.chain(300, seed=1, pin_first=False)
    say("free chain")
    teacher_forced(a, 2)
    b = mi.chain(300, seed=2)
    b.jtype = np.append(b.jtype, 0).astype(np.uint8)
    b.ja = np.append(b.ja, -1).astype(np.int32)
    b.jb = np.append(b.jb, 299).astype(np.int32)
    tip = b.q0[299, 9:] + np.array([0.5, 0, 0])
    b.pa = np.vstack([b.pa, tip]); b.pb = np.vstack([b.pb, [0.5, 0, 0]])
    b.axis = np.vstack([b.axis, [0, 1, 0]]); b.cp_len = np.append(b.cp_len, 0.1)
    say("chain with world end")
    teacher_forced(b, 2)
    c = mi.chain(300, seed=3)
    sw = np.arange(0, 299, 2)
    c.ja[sw], c.jb[sw] = c.jb[sw].copy(), c.ja[sw].copy()
    c.pa[sw], c.pb[sw] = c.pb[sw].copy(), c.pa[sw].copy()
    say("chain with reversed joints")
    teacher_forced(c, 2)
    d = mi.chain(300, seed=4)
    perm = np.random.default_rng(0).permutation(d.m)
    for f in ("jtype", "ja", "jb", "pa", "pb", "axis", "cp_len"):
        setattr(d, f, getattr(d, f)[perm])
    say("chain with shuffled joint order")
    teacher_forced(d, 2)


def test_tree_and_hinge_paths():
    t = mi.tree(300, seed=5)
    t.qd0[1:] = np.random.default_rng(5).normal(0, 0.05, (299, 12))
    say("tree 300")
    say("worst", teacher_forced(t, 3, tol_v=TOL_V_TREE))
    h = mi.chain(200, seed=6, hinge_frac=0.5)
    say("hinge chain 200")
    say("worst", teacher_forced(h, 3))
    w = mi.tree(100, seed=7, window=3)
    say("tree frozen hinge gradient")
    say("worst", teacher_forced(w, 2, hinge_grad=2, tol_v=TOL_V_TREE))


def test_deep_hinge_chain_contraction():
    """3,000 hinge-jointed links: a path of 5-row blocks, eliminated almost
    entirely by compress rounds of the tree contraction (the path solver off;
    tests/test_gpu_paths.py covers it)."""
    asm = mi.chain(3000, seed=41, hinge_frac=1.0)
    asm.qd0[1:] = np.random.default_rng(41).normal(0, 0.05, (asm.n - 1, 12))
    say("all-hinge chain 3000")
    say("worst", teacher_forced(asm, 2, tol_v=TOL_V_TREE, path_solver=0))


def test_wide_tree_contraction():
    """8-ary tree: every interior body absorbs 8 child joints (cliques of up
    to 45 rows), so rakes dominate and the large-clique storage is used."""
    n = 600
    parents = np.array([0] + [(i - 1) // 8 for i in range(1, n)])
    asm = mi.tree(n, seed=42, parents=parents)
    asm.qd0[1:] = np.random.default_rng(42).normal(0, 0.05, (n - 1, 12))
    say("8-ary tree", n)
    say("worst", teacher_forced(asm, 2, tol_v=TOL_V_TREE))


def test_largest_clique_rake():
    """Hinge tree below a pinned body 0 and one link (body 1): bodies 2-12
    each carry eleven 5-row leaf joints under a 5-row parent joint, so they
    are raked with cliques of 60 rows (the largest LDS-staged class, within
    4 of the 64-row limit) and the partial Cholesky's trailing triangles are
    wider than half a wave; body 1 ends with a 60-row root clique."""
    parents = np.array([0, 0] + [1] * 11 + [2 + j // 11 for j in range(121)])
    n = len(parents)
    asm = mi.tree(n, seed=49, parents=parents, hinge_frac=1.0)
    asm.qd0[1:] = np.random.default_rng(49).normal(0, 0.05, (n - 1, 12))
    say("11-ary hinge tree", n)
    say("worst", teacher_forced(asm, 2, tol_v=TOL_V_TREE))


def test_large_clique_compress():
    """A body with ten hinge leaves and one hinge child chain, under a short
    chain: after the leaves are raked it has a single live child, so it is
    compressed with a 60-row clique, larger than the LDS-staged kernels take
    (the team kernels on the global slots run it)."""
    parents = np.array([0, 0, 1, 2, 3, 4] + [5] * 10 + [5] + list(range(16, 60)))
    asm = mi.tree(len(parents), seed=48, parents=parents, hinge_frac=1.0)
    asm.qd0[1:] = np.random.default_rng(48).normal(0, 0.05, (asm.n - 1, 12))
    say("60-row clique compress, bodies", asm.n)
    say("worst", teacher_forced(asm, 2, tol_v=TOL_V_TREE))


def test_many_tree_components():
    """Trees and hinge chains of different depths in one context: their
    contraction rounds run in the same launches."""
    parts = [mi.tree(700, seed=43), mi.chain(400, seed=44, hinge_frac=0.5, origin=(0.0, 15.0, 0.0)),
             mi.tree(40, seed=45, window=2, origin=(0.0, 30.0, 0.0)),
             mi.chain(5, seed=46, hinge_frac=1.0, origin=(0.0, 45.0, 0.0)),
             mi.tree(1500, seed=47, window=4, origin=(0.0, 60.0, 0.0))]
    asm = mi.concat(parts, h=1e-2, steps=2)
    say("mixed trees", asm.n)
    say("worst", teacher_forced(asm, 2, tol_v=TOL_V_TREE))


def test_tree_with_world_joints_and_lame():
    t = mi.tree(120, seed=8, window=8)
    t.jtype = np.append(t.jtype, [0, 1]).astype(np.uint8)
    t.ja = np.append(t.ja, [50, -1]).astype(np.int32)
    t.jb = np.append(t.jb, [-1, 90]).astype(np.int32)
    p50 = t.q0[50, 9:] + np.array([0.0, 0.0, 0.02])
    p90 = t.q0[90, 9:] + np.array([0.0, 0.01, 0.0])
    t.pa = np.vstack([t.pa, [0.0, 0.0, 0.02], p90]); t.pb = np.vstack([t.pb, p50, [0.0, 0.01, 0.0]])
    t.axis = np.vstack([t.axis, [0, 1, 0], [0.6, 0, 0.8]]); t.cp_len = np.append(t.cp_len, [0.1, 0.1])
    t.material = 1
    t.poisson = np.full(t.n, 0.3)
    t.k_orth[:] = 1e8
    say("tree with world joints, Lame material")
    say("worst", teacher_forced(t, 2, tol_v=TOL_V_TREE))


def test_newton_iterations():
    t = mi.tree(60, seed=9)
    t.qd0[1:] = np.random.default_rng(9).normal(0, 0.5, (59, 12))
    say("tree newton 3")
    say("worst", teacher_forced(t, 2, newton_iters=3, tol_v=TOL_V_TREE))


def test_multi_step_call_equals_single_steps():
    asm = mi.chain(600, seed=10)
    a = ctx_of(asm); b = ctx_of(asm)
    a.step(asm.h, 5)
    for _ in range(5):
        b.step(asm.h, 1)
    qa, qda = a.state(); qb, qdb = b.state()
    assert np.array_equal(qa, qb) and np.array_equal(qda, qdb)


def test_state_roundtrip_and_device_copy():
    import torch

    asm = mi.tree(200, seed=11)
    ctx = ctx_of(asm)
    ctx.step(asm.h, 3)
    q, qd = ctx.state()
    ctx.set_state(q, qd)
    ctx.step(asm.h, 2)
    q1, qd1 = ctx.state()
    ref = ctx_of(asm)
    ref.step(asm.h, 5)
    q2, qd2 = ref.state()
    assert np.array_equal(q1, q2) and np.array_equal(qd1, qd2)
    tq = torch.zeros((asm.n, 12), dtype=torch.float64, device="cuda")
    tqd = torch.zeros((asm.n, 12), dtype=torch.float64, device="cuda")
    ctx.state_device(tq, tqd)
    torch.cuda.synchronize()
    assert np.array_equal(tq.cpu().numpy(), q1) and np.array_equal(tqd.cpu().numpy(), qd1)
    assert np.array_equal(q1[0], asm.q0[0]) and np.all(qd1[0] == 0.0)


def test_nonfinite_step_keeps_last_state():
    import paper_2603_08079_amd as pk

    asm = mi.chain(40, seed=12)
    ctx = ctx_of(asm)
    ctx.step(asm.h, 2)
    q, qd = ctx.state()
    bad = qd.copy()
    bad[5, 9] = 1e308
    ctx.set_state(q, bad)
    ctx.step(asm.h, 3)  # queued: mabd_state reads the outcome
    with pytest.raises(pk.MabdError) as ei:
        ctx.state()
    assert ei.value.status == pk.ERR_NONFINITE
    q1, qd1 = ctx.state()
    assert np.array_equal(q1, q) and np.array_equal(qd1, bad)


def test_full_size_chain_one_step():
    """The 1,048,576-body chain at full size, in the launch configuration the
    benchmark times: one step from a perturbed moving state, compared body by
    body with the oracle (block Thomas over all 1,048,575 rows)."""
    asm = mi.config("chain1m")
    rng = np.random.default_rng(20)
    asm.qd0[1:, 9:] = rng.normal(0, 0.05, (asm.n - 1, 3))
    say("chain1m full size")
    ctx = ctx_of(asm)
    ctx.step(asm.h, 1)
    qg, qdg = ctx.state()
    lam_g = ctx.multipliers()
    s = oracle.System(asm)
    q1, qd1, lam, d = s.step(asm.h, asm.q0, asm.qd0)
    eq, eqd = state_errors(qg, qdg, q1, qd1)
    el = rel_err(lam_g, lam, 1.0)
    say("errors", eq, eqd, el, "oracle kkt", d[:3])
    assert eq < TOL and eqd < TOL and el < 1e-8
    # the GPU multipliers satisfy the FP64 KKT system to the oracle's level
    qv, qdv, dv = s.finish(asm.h, asm.q0, asm.qd0, lam_g)
    say("kkt of GPU multipliers", dv[:3])
    assert dv[oracle.KKT] < 1e-12


def test_full_size_tree_one_step():
    """The 262,144-body random tree (ball/hinge 50/50, ~8,000 levels)."""
    asm = mi.config("tree256k")
    say("tree256k full size")
    ctx = ctx_of(asm)
    ctx.step(asm.h, 1)
    qg, qdg = ctx.state()
    s = oracle.System(asm)
    q1, qd1, lam, d = s.step_sparse(asm.h, asm.q0, asm.qd0)
    eq, eqd = state_errors(qg, qdg, q1, qd1)
    say("errors", eq, eqd, "oracle kkt", d[:3])
    qv, qdv, dv = s.finish(asm.h, asm.q0, asm.qd0, ctx.multipliers())
    say("kkt of GPU multipliers", dv[:3])
    assert eq < TOL and eqd < TOL_V_TREE
    assert dv[oracle.KKT] <= max(10 * d[oracle.KKT], 1e-11)


def part_of(asm, b0, b1):
    """Bodies [b0, b1) of an assembly of independent parts, with their joints
    (indices shifted), as an assembly of its own."""
    import dataclasses

    jm = ((asm.ja >= b0) & (asm.ja < b1)) | ((asm.jb >= b0) & (asm.jb < b1))
    shift = lambda x: np.where(x >= 0, x - b0, -1).astype(np.int32)
    return dataclasses.replace(
        asm, name=f"{asm.name}[{b0}:{b1}]", dims=asm.dims[b0:b1], density=asm.density[b0:b1],
        k_orth=asm.k_orth[b0:b1], pinned=asm.pinned[b0:b1], q0=asm.q0[b0:b1], qd0=asm.qd0[b0:b1],
        poisson=None if asm.poisson is None else asm.poisson[b0:b1], jtype=asm.jtype[jm],
        ja=shift(asm.ja[jm]), jb=shift(asm.jb[jm]), pa=asm.pa[jm], pb=asm.pb[jm], axis=asm.axis[jm],
        cp_len=asm.cp_len[jm], meta={})


def test_full_size_batch_one_step():
    """The 4,096-assembly batch (2.95M bodies, chains and trees, ball/hinge
    50/50) at full size, in the launch configuration the benchmark times (one
    context, graph replay): the FP64 KKT residual of the GPU multipliers over
    the whole batch, and nine assemblies (the smallest, the largest, the
    largest tree, the first four and two drawn at random) body by body against
    the oracle's own step of that assembly alone."""
    asm = mi.config("batch4096")
    say("batch4096 full size", asm.n, asm.m)
    ctx = ctx_of(asm)
    ctx.step(asm.h, 1)
    assert ctx.stats()["graph_replay"] == 1
    qg, qdg = ctx.state()
    lam_g = ctx.multipliers()
    ctx.close()
    s = oracle.System(asm)
    _, _, dv = s.finish(asm.h, asm.q0, asm.qd0, lam_g)
    say("kkt of GPU multipliers over the batch", dv[:3])
    sizes = np.asarray(asm.meta["sizes"])
    off = np.concatenate([[0], np.cumsum(sizes)])
    tree_sizes = np.where(np.asarray(asm.meta["chain"]), -1, sizes)
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.argmax(tree_sizes)), 0, 1, 2, 3,
                    *np.random.default_rng(49).choice(len(sizes), 2, replace=False).tolist()})
    worst_kkt = 0.0
    for i in picks:
        sub = part_of(asm, off[i], off[i + 1])
        sp = oracle.System(sub)
        q1, qd1, lam, d = reference_step(sp, sub, sub.q0, sub.qd0, oracle.AUTO)
        eq, eqd = state_errors(qg[off[i]:off[i + 1]], qdg[off[i]:off[i + 1]], q1, qd1)
        worst_kkt = max(worst_kkt, d[oracle.KKT])
        say(f"  part {i} ({'chain' if asm.meta['chain'][i] else 'tree'}, {sub.n} bodies): errors", eq, eqd,
            "oracle kkt", d[oracle.KKT])
        assert eq < TOL and eqd < TOL_V_TREE, (i, eq, eqd)
    assert dv[oracle.KKT] <= max(10 * worst_kkt, 1e-11)


def test_full_size_lattice_one_step():
    """The 512 x 512 lattice (522,753 ball joints closing loops) at full size:
    one cold-start PCG step to 1e-10; the oracle's FP64 dual residual of the
    GPU multipliers must be at that tolerance (a direct factorisation of this
    system is too large to serve as the reference state)."""
    asm = mi.config("lattice512")
    say("lattice512 full size", asm.n, asm.m)
    ctx = ctx_of(asm, kkt_tol=1e-10, warm_start=0)
    ctx.step(asm.h, 1)
    st = ctx.stats()
    lam_g = ctx.multipliers()
    qg, qdg = ctx.state()
    ctx.close()
    s = oracle.System(asm)
    qv, qdv, dv = s.finish(asm.h, asm.q0, asm.qd0, lam_g)
    say("pcg iterations", st["pcg_iters"], "kkt of GPU multipliers", dv[:3])
    assert dv[oracle.RHO_D] <= 2e-10 and dv[oracle.RHO_P] <= 1e-12
    # the GPU's back-projection of its multipliers is the oracle's
    eq, eqd = state_errors(qg, qdg, qv, qdv)
    say("state vs the oracle's back-projection of the GPU multipliers", eq, eqd)
    assert eq < TOL and eqd < TOL


def test_full_size_rgg_one_step():
    """The 100,000-body random geometric network (244,291 ball joints, six
    network components, five of them with few enough loops for the
    loop-breaker, and twelve trees) at full size: one cold-start PCG
    step to relative residual 1e-2, a tolerance block-Jacobi PCG reaches on
    this over-constrained graph within a few thousand iterations (1e-10 is
    out of its reach).  The oracle back-projects the GPU multipliers in FP64
    and must find the dual residual at that tolerance and the primal one at
    rounding level."""
    tol = 1e-2
    asm = mi.config("rgg100k")
    say("rgg100k full size", asm.n, asm.m)
    ctx = ctx_of(asm, kkt_tol=tol, max_iters=100000, warm_start=0)
    ctx.step(asm.h, 1)
    st = ctx.stats()
    lam_g = ctx.multipliers()
    qg, qdg = ctx.state()
    ctx.close()
    # six network components: the five with few loops are solved exactly by
    # the loop-breaker, the large one by PCG
    assert st["n_graph"] + st["n_loop"] == 6 and st["n_graph"] >= 1 and st["last_status"] == 0
    assert 0 < st["pcg_iters"] < 100000 and st["rho_d"] <= tol
    s = oracle.System(asm)
    qv, qdv, dv = s.finish(asm.h, asm.q0, asm.qd0, lam_g)
    say("pcg iterations", st["pcg_iters"], "GPU residual", st["rho_d"], "kkt of GPU multipliers", dv[:3])
    assert dv[oracle.RHO_D] <= 2 * tol and dv[oracle.RHO_P] <= 1e-12
    # the GPU's back-projection of its multipliers is the oracle's
    eq, eqd = state_errors(qg, qdg, qv, qdv)
    say("state vs the oracle's back-projection of the GPU multipliers", eq, eqd)
    assert eq < TOL and eqd < TOL
    # the GPU's own true residual of the PCG network and the oracle's over
    # all rows (the other components' rows are solved exactly) are the same
    # number up to the share of the exactly solved rows in the norm of r
    assert abs(dv[oracle.RHO_D] - st["rho_d"]) <= 1e-2 * st["rho_d"]
