"""Captured step graphs and the chain tile-size autotuner.

A context with no PCG component replays each step as a captured hipGraph (one
per state-buffer parity).  The replays must give bit-identical results to the
eager launch sequence, across calls, step counts, a change of h and eager work
queued between replays; the autotuned tile size must give the oracle's step.
"""
import numpy as np
import pytest

import mabd_inputs as mi
import oracle
from gpu_util import say, state_errors

pytestmark = pytest.mark.gpu


def mixed_assembly():
    parts = [mi.chain(3000, seed=31), mi.chain(500, seed=32, hinge_frac=0.5, origin=(0.0, 30.0, 0.0)),
             mi.tree(300, seed=33, origin=(0.0, -30.0, 0.0))]
    return mi.concat(parts, h=1e-2, steps=4)


def test_graph_replay_matches_eager():
    import torch
    import paper_2603_08079_amd as pk

    asm = mixed_assembly()
    stream = torch.cuda.Stream()
    g = pk.Context(asm, stream=stream.cuda_stream, use_graph=1)
    e = pk.Context(asm, stream=stream.cuda_stream, use_graph=0)
    assert g.stats()["n_graph"] == 0
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for n, h in [(1, 1e-2), (3, 1e-2), (2, 5e-3), (1, 1e-2), (4, 1e-2)]:
        g.step(h, n)
        assert g.stats()["graph_replay"] == 1
        with torch.cuda.stream(stream):  # eager work between replays, same stream
            scratch.add_(1.0)
            scratch.mul_(0.5)
        e.step(h, n)
        assert e.stats()["graph_replay"] == 0
        qg, qdg = g.state()
        qe, qde = e.state()
        say("steps", n, "h", h, "max |dq|", np.abs(qg - qe).max(), "max |dqd|", np.abs(qdg - qde).max())
        assert np.array_equal(qg, qe) and np.array_equal(qdg, qde)
        assert np.array_equal(g.multipliers(), e.multipliers())
    torch.cuda.synchronize()
    assert g.stats()["steps_done"] == e.stats()["steps_done"] == 11


def test_graph_state_device_on_caller_stream():
    import torch
    import paper_2603_08079_amd as pk

    asm = mi.chain(2000, seed=34)
    stream = torch.cuda.Stream()
    ctx = pk.Context(asm, stream=stream.cuda_stream)
    ref = pk.Context(asm, use_graph=0)
    tq = torch.empty((asm.n, 12), dtype=torch.float64, device="cuda")
    tqd = torch.empty_like(tq)
    for _ in range(3):
        ctx.step(asm.h, 2)
        ref.step(asm.h, 2)
        ctx.state_device(tq, tqd)
        with torch.cuda.stream(stream):
            hq = tq.cpu().numpy()
            hqd = tqd.cpu().numpy()
        qr, qdr = ref.state()
        assert np.array_equal(hq, qr) and np.array_equal(hqd, qdr)


def test_graph_nonfinite_rollback():
    import paper_2603_08079_amd as pk

    asm = mi.chain(100, seed=35)
    ctx = pk.Context(asm)
    ctx.step(asm.h, 3)
    q, qd = ctx.state()
    bad = qd.copy()
    bad[50, 10] = 1e308  # finite input whose step overflows
    ctx.set_state(q, bad)
    ctx.step(asm.h, 4)  # queued: the outcome is read by the next call
    st = ctx.stats()
    assert st["last_status"] == pk.ERR_NONFINITE and st["graph_replay"] == 1
    q1, qd1 = ctx.state()
    assert np.array_equal(q1, q) and np.array_equal(qd1, bad)
    # the context keeps working after the failure
    ctx.set_state(q, qd)
    ctx.step(asm.h, 2)
    ref = pk.Context(asm, use_graph=0)
    ref.set_state(q, qd)
    ref.step(asm.h, 2)
    qa, qda = ctx.state()
    qb, qdb = ref.state()
    assert np.array_equal(qa, qb) and np.array_equal(qda, qdb)


def test_autotuned_tiles_match_oracle():
    import paper_2603_08079_amd as pk

    asm = mi.chain(40000, seed=36)
    rng = np.random.default_rng(37)
    asm.qd0[1:, 9:] = rng.normal(0, 0.05, (asm.n - 1, 3))
    tuned = pk.Context(asm, autotune=1)
    fixed = pk.Context(asm, autotune=0)
    tuned.step(asm.h, 1)
    fixed.step(asm.h, 1)
    tt = tuned.stats()["tile_threads"]
    say("autotuned tile threads", tt)
    assert tt in (64, 128, 256) and fixed.stats()["tile_threads"] == 64
    s = oracle.System(asm)
    q1, qd1, lam, d = s.step(asm.h, asm.q0, asm.qd0)
    for ctx in (tuned, fixed):
        qg, qdg = ctx.state()
        eq, eqd = state_errors(qg, qdg, q1, qd1)
        say("vs oracle", eq, eqd)
        assert eq < 1e-10 and eqd < 1e-10


@pytest.mark.parametrize("tt", ["64p", "64", "128", "256"])
def test_forced_tile_size(tt, monkeypatch):
    """MABD_CHAIN_TILE_THREADS fixes the tile size at create (no autotuning);
    "64p" selects the packed 60-row tiles."""
    import paper_2603_08079_amd as pk

    monkeypatch.setenv("MABD_CHAIN_TILE_THREADS", tt)
    asm = mi.chain(5000, seed=38)
    ctx = pk.Context(asm)
    st = ctx.stats()
    assert st["tile_threads"] == int(tt.rstrip("p"))
    assert st["tile_packed"] == (1 if tt.endswith("p") else 0)
    ctx.step(asm.h, 2)
    q, qd = asm.q0, asm.qd0
    s = oracle.System(asm)
    for _ in range(2):
        q, qd, lam, d = s.step(asm.h, q, qd)
    qg, qdg = ctx.state()
    eq, eqd = state_errors(qg, qdg, q, qd)
    say("tile threads", tt, eq, eqd)
    assert eq < 1e-10 and eqd < 1e-10
