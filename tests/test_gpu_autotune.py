"""Autotuner and tuning cache on the GPU: the tree schedules it times (split
threshold of the 16-row cliques, class order within a launch) change no
result, so a tuned context's state is bitwise the untuned one's; a context
that times its schedules appends them to the tuning cache, and a second
context of the same shape takes them from the file without timing."""
import numpy as np
import pytest

import mabd_inputs as mi
from gpu_util import say

pytestmark = pytest.mark.gpu

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

SPLITS = (1500, 6000, 2**31 - 1)


def tree_and_chain():
    """A 24,000-body tree (enough slots for the tree tuner) beside a
    7,000-body ball chain (21,000 chain rows, enough for the chain tuner)."""
    t = mi.tree(24000, seed=141)
    c = mi.chain(7000, seed=142, origin=(0.0, 50.0, 0.0))
    a = mi.concat([t, c], h=1e-2, steps=3)
    a.qd0[:] = np.random.default_rng(143).normal(0, 0.05, a.qd0.shape)
    a.qd0[a.pinned == 1] = 0.0
    return a


def run(asm, steps, **kw):
    import paper_2603_08079_amd as pk

    ctx = pk.Context(asm, **kw)
    st0 = ctx.stats()
    ctx.step(asm.h, steps)
    q, qd = ctx.state()
    st = ctx.stats()
    ctx.close()
    return q, qd, st0, st


def test_tuned_schedule_changes_no_result():
    asm = tree_and_chain()
    q0, qd0, _, s0 = run(asm, 2, autotune=0)
    q1, qd1, _, s1 = run(asm, 2, autotune=1)
    say("untuned", s0["tree_split"], s0["tree_order"], s0["tile_threads"], s0["tile_packed"],
        "tuned", s1["tree_split"], s1["tree_order"], s1["tile_threads"], s1["tile_packed"])
    assert s0["tune_source"] == 0 and s1["tune_source"] == 1
    assert s0["tree_split"] == 6000 and s0["tree_order"] == 0
    assert s1["tree_split"] in SPLITS and s1["tree_order"] in (0, 1)
    assert s1["last_status"] == 0 and s1["steps_done"] == 2
    # tile forms reduce the chain in a different order; the tree schedules do not
    if s1["tile_threads"] == 64 and s1["tile_packed"] == 1:
        assert np.array_equal(q0, q1) and np.array_equal(qd0, qd1)
    else:
        assert np.abs(q0 - q1).max() <= 1e-10 * np.abs(q0).max()


def test_every_tree_schedule_gives_the_same_state():
    """Pinning each schedule through the cache file: bitwise equal states."""
    asm = mi.tree(24000, seed=144)
    asm.qd0[1:] = np.random.default_rng(145).normal(0, 0.05, (asm.n - 1, 12))
    import paper_2603_08079_amd as pk
    import tempfile, os

    ref = None
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        # the key of this shape, from a context that times its schedules
        ctx = pk.Context(asm, autotune=1, tune_cache=path)
        ctx.step(asm.h, 1)
        ctx.close()
        key = open(path).read().split(" = ")[0]
        for split in SPLITS:
            for order in (0, 1):
                with open(path, "w") as f:
                    f.write(f"{key} = 64 1 {split} {order}\n")
                q, qd, st0, st = run(asm, 2, autotune=1, tune_cache=path)
                assert st0["tune_source"] == 2 and st["tree_split"] == split and st["tree_order"] == order
                if ref is None:
                    ref = (q, qd)
                assert np.array_equal(q, ref[0]) and np.array_equal(qd, ref[1]), (split, order)
    say("six schedules, one state")


def test_tuning_cache_round_trip(tmp_path):
    asm = tree_and_chain()
    path = str(tmp_path / "tune.txt")
    q1, qd1, a0, a = run(asm, 2, autotune=1, tune_cache=path)
    lines = open(path).read().splitlines()
    say("cache", lines)
    assert a0["tune_source"] == 0 and a["tune_source"] == 1 and len(lines) == 1
    key, val = lines[0].split(" = ")
    assert "gfx" in key and val.split() == [str(a["tile_threads"]), str(a["tile_packed"]),
                                            str(a["tree_split"]), str(a["tree_order"])]
    q2, qd2, b0, b = run(asm, 2, autotune=1, tune_cache=path)
    assert b0["tune_source"] == 2 and b["tune_source"] == 2
    for f in ("tile_threads", "tile_packed", "tree_split", "tree_order"):
        assert a[f] == b[f], f
    assert np.array_equal(q1, q2) and np.array_equal(qd1, qd2)
    assert len(open(path).read().splitlines()) == 1  # nothing timed, nothing appended
    # another shape (one body fewer in the tree) has no entry: timed, appended
    other = mi.concat([mi.tree(23999, seed=141), mi.chain(7000, seed=142, origin=(0.0, 50.0, 0.0))],
                      h=1e-2, steps=3)
    _, _, c0, c = run(other, 1, autotune=1, tune_cache=path)
    assert c["tune_source"] == 1 and len(open(path).read().splitlines()) == 2


def test_malformed_cache_entries_are_ignored(tmp_path):
    asm = mi.tree(24000, seed=146)
    path = str(tmp_path / "tune.txt")
    run(asm, 1, autotune=1, tune_cache=path)
    key = open(path).read().split(" = ")[0]
    with open(path, "w") as f:
        f.write(f"{key} = 96 1 6000 0\n{key} = 64 1 -5 0\n{key} = 64 1\ngarbage\n")
    _, _, s0, s = run(asm, 1, autotune=1, tune_cache=path)
    assert s0["tune_source"] == 0 and s["tune_source"] == 1
    # a missing directory: timed, the append fails quietly
    _, _, _, s = run(asm, 1, autotune=1, tune_cache=str(tmp_path / "no" / "such" / "dir.txt"))
    assert s["tune_source"] == 1 and s["last_status"] == 0
