"""The polar-free single-body solve (Alg. 1, body_solve = 1) on the GPU
against the oracle's: unjointed boxes, rotated, spinning, deformed and loaded
by wrenches, next to jointed assemblies that keep the polar solve, in one
context; and its speed against the polar solve on a million boxes."""
import time

import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors

pytestmark = pytest.mark.gpu

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None


def mixed_scene():
    boxes = mi.spinning_boxes(3000, seed=111)
    rng = np.random.default_rng(112)
    # deform the boxes a little: A = R (I + e N), e ~ 1e-4
    for b in range(boxes.n):
        A = boxes.q0[b, :9].reshape(3, 3).T @ (np.eye(3) + 1e-4 * rng.normal(size=(3, 3)))
        boxes.q0[b, :9] = A.T.reshape(9)
    chain = mi.chain(300, seed=113, hinge_frac=0.3, origin=(0.0, -50.0, 0.0))
    chain.qd0[1:] = rng.normal(0, 0.05, (chain.n - 1, 12))
    tree = mi.tree(200, seed=114, origin=(0.0, -80.0, 0.0))
    return mi.concat([boxes, chain, tree], h=1e-2, steps=3)


def test_polar_free_parity():
    import paper_2603_08079_amd as pk

    asm = mixed_scene()
    W = np.random.default_rng(115).normal(0, 0.5, (asm.n, 6))
    s = oracle.System(asm, body_solve=1, wrench=W)
    ctx = pk.Context(asm, body_solve=1)
    ctx.set_wrenches(W)
    q, qd = asm.q0.copy(), asm.qd0.copy()
    for n in range(3):
        ctx.set_state(q, qd)
        ctx.step(asm.h, 1)
        qg, qdg = ctx.state()
        q1, qd1, lam, d = s.step(asm.h, q, qd)
        eq, eqd = state_errors(qg, qdg, q1, qd1)
        say(n, "polar-free scene errors", eq, eqd)
        assert eq < 1e-10 and eqd < 1e-10
        q, qd = q1, qd1
    # the polar-free solve is a different step from the polar one
    s0 = oracle.System(asm, wrench=W)
    q0, qd0, _, _ = s0.step(asm.h, asm.q0, asm.qd0)
    qf, qdf, _, _ = s.step(asm.h, asm.q0, asm.qd0)
    assert np.abs(qdf[:3000] - qd0[:3000]).max() > 1e-12 * np.abs(qd0).max()
    assert np.array_equal(qf[3000:], q0[3000:])


def test_polar_free_speed_on_a_million_boxes():
    """Per-step time of the polar and polar-free solves on 1,048,576 spinning
    boxes (reported; the polar-free step must not be slower)."""
    import paper_2603_08079_amd as pk

    asm = mi.config("boxes1m")
    times = {}
    for bs in (0, 1):
        ctx = pk.Context(asm, body_solve=bs)
        ctx.step(asm.h, 2)
        ctx.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(asm.h, 20)
        ctx.stats()
        times[bs] = (time.perf_counter() - t0) / 20 * 1e3
        ctx.close()
    say("ms per step: polar", times[0], "polar-free", times[1])
    assert times[1] <= 1.05 * times[0]


@pytest.mark.parametrize("body_solve", [0, 1])
def test_fused_back_projection_of_free_bodies(body_solve):
    """Bodies without joints take their back-projection in the body kernel,
    except where every Newton iteration's residual is recorded (diagnostics
    with several iterations keep the separate kernel): both give the same
    state bitwise, beside jointed assemblies, over two iterations a step."""
    import paper_2603_08079_amd as pk

    asm = mixed_scene()
    out = []
    for diag in (0, 1):
        ctx = pk.Context(asm, body_solve=body_solve, newton_iters=2, diagnostics=diag)
        ctx.step(asm.h, 3)
        q, qd = ctx.state()
        st = ctx.stats()
        ctx.close()
        assert st["last_status"] == 0
        out.append((q, qd))
    say("body_solve", body_solve, "max |q|", np.abs(out[0][0]).max())
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("body_solve", [0, 1])
def test_full_size_boxes_sampled(body_solve):
    """The 1,048,576 spinning boxes as the benchmark runs them, two steps;
    the bodies are independent, so a sample of 2,000 of them stepped by the
    oracle alone must match the GPU's state of the same bodies."""
    import paper_2603_08079_amd as pk

    asm = mi.config("boxes1m")
    ctx = pk.Context(asm, body_solve=body_solve)
    ctx.step(asm.h, 2)
    qg, qdg = ctx.state()
    ctx.close()
    idx = np.sort(np.random.default_rng(131).choice(asm.n, 2000, replace=False))
    sub = mi.spinning_boxes(1, seed=0)  # template of an unjointed assembly
    sub.dims, sub.density, sub.k_orth = asm.dims[idx], asm.density[idx], asm.k_orth[idx]
    sub.pinned, sub.q0, sub.qd0 = asm.pinned[idx], asm.q0[idx], asm.qd0[idx]
    if asm.poisson is not None:
        sub.poisson = asm.poisson[idx]
    s = oracle.System(sub, body_solve=body_solve)
    q, qd = sub.q0.copy(), sub.qd0.copy()
    for _ in range(2):
        q, qd, _, _ = s.step(asm.h, q, qd)
    eq, eqd = state_errors(qg[idx], qdg[idx], q, qd)
    say("boxes1m body_solve", body_solve, "sampled errors", eq, eqd)
    assert eq < 1e-10 and eqd < 1e-10
