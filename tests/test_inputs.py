"""Shapes and counts of the seeded synthetic workloads."""
import numpy as np

import mabd_inputs as mi
import oracle


def test_chain_config_shape():
    a = mi.config("chain64")
    assert a.n == 64 and a.m == 63 and a.rows() == 189
    assert a.pinned[0] == 1 and a.pinned[1:].sum() == 0
    assert np.all(a.jtype == 0)
    s = oracle.System(a)
    assert s.classify() == 1
    # anchors sit at the midpoint of the perturbed end centres: C(q0) = 0
    for k in range(a.m):
        C, _, _ = s.joint_terms(a.q0, k)
        assert np.abs(C).max() < 1e-14


def test_tree_generator_depth_and_mix():
    a = mi.tree(4096, seed=0)
    par = a.meta["parent"]
    depth = np.zeros(a.n, int)
    for i in range(1, a.n):
        depth[i] = depth[par[i]] + 1
    assert depth.max() > 100                     # deep, narrow tree
    assert 0.4 < a.jtype.mean() < 0.6            # ball/hinge 50/50
    assert np.all((a.dims >= 0.05) & (a.dims <= 0.5))
    assert oracle.System(a).classify() == 2


def test_batch_sizes_log_uniform():
    a = mi.batch(64, seed=1)
    sizes = np.asarray(a.meta["sizes"])
    assert sizes.min() >= 16 and sizes.max() <= 4096 and a.n == sizes.sum()
    assert a.pinned.sum() == len(sizes)


def test_lattice_and_rgg_counts():
    a = mi.lattice(8, seed=0)
    assert a.n == 64 and a.m == 2 * 8 * 7 - 7
    assert oracle.System(a).classify() == 3
    g = mi.rgg(2000, seed=0)
    deg = np.bincount(np.concatenate([g.ja, g.jb]), minlength=g.n)
    assert 1.5 < g.m / g.n < 3.5 and deg.max() <= 12
    assert g.pinned.sum() == 20


def test_seeds_reproduce():
    a = mi.tree(300, seed=5)
    b = mi.tree(300, seed=5)
    assert np.array_equal(a.q0, b.q0) and np.array_equal(a.pa, b.pa)
