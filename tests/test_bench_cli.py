"""bench.py on the CPU: more than one GPU is refused with a message before
anything touches a device; the algorithmic bytes of the generic kernel
groups count only the bodies and joints outside the fused chain path."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_generic_parts_leave_out_the_ball_chains():
    """The roofline of a generic kernel group counts the bodies and joints
    outside the fused chain path: a ball chain is left out, a hinge chain, a
    tree and a single body held by one ball joint (one joint: not a chain)
    stay in; pinned bodies are never counted."""
    sys.path.insert(0, ROOT)
    import mabd_inputs as mi
    import bench

    parts = [mi.chain(10, seed=1), mi.chain(8, seed=2, hinge_frac=1.0, origin=(0.0, 10.0, 0.0)),
             mi.tree(12, seed=3, origin=(0.0, 20.0, 0.0)), mi.chain(2, seed=4, origin=(0.0, 30.0, 0.0))]
    a = mi.concat(parts)
    bm, jm = bench.generic_parts(a)
    nb = [p.n for p in parts]
    nj = [p.m for p in parts]
    bo = np.concatenate([[0], np.cumsum(nb)])
    jo = np.concatenate([[0], np.cumsum(nj)])
    assert not bm[bo[0]:bo[1]].any() and not jm[jo[0]:jo[1]].any()      # ball chain
    for i in (1, 2, 3):
        pinned = np.asarray(a.pinned[bo[i]:bo[i + 1]]) == 1
        assert (bm[bo[i]:bo[i + 1]] == ~pinned).all() and jm[jo[i]:jo[i + 1]].all()
    # the bytes of the tree group follow the masks
    t = bench.generic_alg_bytes(a, "tree")
    sub = mi.concat(parts[1:])
    assert t == bench.generic_alg_bytes(sub, "tree")
