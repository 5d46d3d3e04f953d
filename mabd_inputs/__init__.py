"""Seeded synthetic assemblies shaped like the paper's workloads.

This module builds *inputs only* (geometry, masses, joint anchors, initial
state) with ``numpy.random.default_rng``.  It holds none of the method's
arithmetic: no polar decomposition, no Hessians, no constraint rows.  It is the
one piece shared by the FP64 oracle and the GPU library's tests/benchmarks.

Layout conventions (paper Sec. 3.1 and Sec. 4.1):
  * q per body = [a1; a2; a3; t] (12 doubles), a_c the c-th column of A;
  * a joint is (type, a, b, pa, pb, axis, cp_len, axis2): type 0 ball (Eq.
    ball), 1 five-row hinge (Eq. hinge), 2 four-row universal (Eq. universal),
    3 five-row prismatic (Eq. prismatic); a/b body indices (-1 = world); pa/pb
    the first control point in each body's rest frame; axis the hinge or
    prismatic axis, or the universal joint's first axis, in a's rest frame;
    axis2 the universal joint's second axis (orthogonal to the first, a's
    rest frame); cp_len the spacing of the further control points.

Workloads (the paper's scenes are not reproducible: their geometry is not
published, so these stand in for them at the configurations' sizes):
  chain    -- boxes 1.0 x 0.1 x 0.1 m along x, ball joints at end centres,
              body 0 pinned (pulley chain, Sec. 6.3 "Joint chain"); with
              hinge_frac > 0 a share of the joints are hinges (hchain1m);
  tree     -- random tree, parent of body i uniform over the previous `window`
              bodies, ball/hinge 50/50, box edges U(0.05, 0.5) m (Sec. 6.3
              "Joint hierarchy");
  batch    -- thousands of independent chains/trees of log-uniform size;
  lattice  -- 2D net of 0.2 x 0.2 x 0.05 m plates with 4-neighbour ball joints,
              one boundary row pinned (ball-joint nets, Sec. 6.2);
  rgg      -- random geometric graph of 0.2 m cubes, ball joints to at most
              four nearest neighbours within 1.5 m, 1 % pinned.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GRAVITY = (0.0, 0.0, -9.8)
BALL, HINGE, UNIVERSAL, PRISMATIC = 0, 1, 2, 3
JOINT_ROWS = (3, 5, 4, 5)   # constraint rows per joint type


@dataclasses.dataclass
class Assembly:
    name: str
    dims: np.ndarray          # (n, 3) float64
    density: np.ndarray       # (n,)
    k_orth: np.ndarray        # (n,)
    pinned: np.ndarray        # (n,) uint8
    q0: np.ndarray            # (n, 12)
    qd0: np.ndarray           # (n, 12)
    jtype: np.ndarray         # (m,) uint8
    ja: np.ndarray            # (m,) int32
    jb: np.ndarray            # (m,) int32
    pa: np.ndarray            # (m, 3)
    pb: np.ndarray            # (m, 3)
    axis: np.ndarray          # (m, 3)
    cp_len: np.ndarray        # (m,)
    poisson: Optional[np.ndarray] = None
    axis2: Optional[np.ndarray] = None  # (m, 3) universal joints' second axis
    gravity: tuple = GRAVITY
    material: int = 0         # 0 orthogonality stiffness k_A, 1 Lame from (E, nu)
    h: float = 1e-2
    steps: int = 1
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.dims.shape[0])

    @property
    def m(self) -> int:
        return int(self.jtype.shape[0])

    def rows(self) -> int:
        return int(np.asarray(JOINT_ROWS)[self.jtype].sum())

    def copy(self) -> "Assembly":
        return dataclasses.replace(self, **{f.name: (getattr(self, f.name).copy()
                                    if isinstance(getattr(self, f.name), np.ndarray)
                                    else getattr(self, f.name))
                                    for f in dataclasses.fields(self)})


def _identity_q(centres: np.ndarray) -> np.ndarray:
    n = centres.shape[0]
    q = np.zeros((n, 12))
    q[:, 0] = 1.0
    q[:, 4] = 1.0
    q[:, 8] = 1.0
    q[:, 9:12] = centres
    return q


def _unit_sphere(rng, k):
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _joint_arrays(m):
    return (np.zeros(m, np.uint8), np.zeros(m, np.int32), np.zeros(m, np.int32),
            np.zeros((m, 3)), np.zeros((m, 3)), np.tile([0.0, 1.0, 0.0], (m, 1)),
            np.full(m, 0.1))


def _midpoint_anchor(ca, cb, na, nb):
    """Joint point between two perturbed bodies (A = I): midpoint of the two
    nominal attachment points, expressed in each body's rest frame, so that the
    constraint holds exactly at t = 0."""
    wa = ca + na
    wb = cb + nb
    mid = 0.5 * (wa + wb)
    return mid - ca, mid - cb


def chain(n: int, seed: int = 0, sigma: float = 1e-3, hinge_frac: float = 0.0,
          link=(1.0, 0.1, 0.1), density: float = 1000.0, k_orth: float = 1e8,
          h: float = 1e-2, steps: int = 200, pin_first: bool = True,
          origin=(0.0, 0.0, 0.0)) -> Assembly:
    """Chain of n boxes along +x; body i centred at (i + 0.5) * link_x plus
    N(0, sigma^2) per coordinate; joint i joins body i's +x end centre to body
    i+1's -x end centre at the midpoint of the perturbed points."""
    rng = np.random.default_rng(seed)
    lx = link[0]
    centres = np.zeros((n, 3))
    centres[:, 0] = (np.arange(n) + 0.5) * lx
    centres += np.asarray(origin, float)
    centres += rng.normal(0.0, sigma, size=(n, 3))
    m = max(n - 1, 0)
    jt, ja, jb, pa, pb, ax, ell = _joint_arrays(m)
    if m:
        ja[:] = np.arange(m)
        jb[:] = np.arange(1, n)
        half = np.array([0.5 * lx, 0.0, 0.0])
        pa[:], pb[:] = _midpoint_anchor(centres[:-1], centres[1:], half, -half)
        if hinge_frac > 0.0:
            jt[:] = (rng.random(m) < hinge_frac).astype(np.uint8)
            ax[:] = _unit_sphere(rng, m)
    pinned = np.zeros(n, np.uint8)
    if pin_first and n:
        pinned[0] = 1
    return Assembly(
        name=f"chain{n}", dims=np.tile(np.asarray(link, float), (n, 1)),
        density=np.full(n, density), k_orth=np.full(n, k_orth), pinned=pinned,
        q0=_identity_q(centres), qd0=np.zeros((n, 12)), jtype=jt, ja=ja, jb=jb,
        pa=pa, pb=pb, axis=ax, cp_len=ell, h=h, steps=steps,
        meta=dict(kind="chain", seed=seed))


def tree(n: int, seed: int = 0, window: int = 64, sigma: float = 1e-3,
         hinge_frac: float = 0.5, dim_range=(0.05, 0.5), density: float = 1000.0,
         k_orth: float = 1e8, h: float = 1e-2, steps: int = 100,
         origin=(0.0, 0.0, 0.0), parents=None) -> Assembly:
    """Random tree: parent of body i > 0 uniform over [max(0, i - window), i - 1]
    (or the given `parents` array, parents[i] < i); A = I; the child's -x end
    centre meets the parent's +x end centre; body 0 pinned; joint type
    Bernoulli(hinge_frac) hinge, else ball; hinge axes uniform on the sphere."""
    rng = np.random.default_rng(seed)
    dims = rng.uniform(dim_range[0], dim_range[1], size=(n, 3))
    parent = np.full(n, -1, np.int64)
    if n > 1:
        lo = np.maximum(0, np.arange(1, n) - window)
        span = np.arange(1, n) - lo
        parent[1:] = lo + np.floor(rng.random(n - 1) * span).astype(np.int64)
        parent[1:] = np.minimum(parent[1:], np.arange(1, n) - 1)
        if parents is not None:
            parent[1:] = np.asarray(parents, np.int64)[1:]
            assert np.all(parent[1:] < np.arange(1, n)) and np.all(parent[1:] >= 0)
    centres = np.zeros((n, 3))
    centres[0] = origin
    for i in range(1, n):
        p = parent[i]
        centres[i] = centres[p] + np.array([0.5 * dims[p, 0] + 0.5 * dims[i, 0], 0.0, 0.0])
    centres += rng.normal(0.0, sigma, size=(n, 3))
    m = max(n - 1, 0)
    jt, ja, jb, pa, pb, ax, ell = _joint_arrays(m)
    if m:
        ja[:] = parent[1:]
        jb[:] = np.arange(1, n)
        hp = np.zeros((m, 3))
        hp[:, 0] = 0.5 * dims[parent[1:], 0]
        hc = np.zeros((m, 3))
        hc[:, 0] = -0.5 * dims[1:, 0]
        pa[:], pb[:] = _midpoint_anchor(centres[parent[1:]], centres[1:], hp, hc)
        jt[:] = (rng.random(m) < hinge_frac).astype(np.uint8)
        ax[:] = _unit_sphere(rng, m)
    pinned = np.zeros(n, np.uint8)
    if n:
        pinned[0] = 1
    return Assembly(
        name=f"tree{n}", dims=dims, density=np.full(n, density),
        k_orth=np.full(n, k_orth), pinned=pinned, q0=_identity_q(centres),
        qd0=np.zeros((n, 12)), jtype=jt, ja=ja, jb=jb, pa=pa, pb=pb, axis=ax,
        cp_len=ell, h=h, steps=steps,
        meta=dict(kind="tree", seed=seed, parent=parent))


def perpendicular(axis):
    """A unit vector orthogonal to each row of `axis` (m x 3)."""
    axis = np.asarray(axis, float).reshape(-1, 3)
    e = np.where(np.abs(axis[:, :1]) < 0.9, [[1.0, 0.0, 0.0]], [[0.0, 1.0, 0.0]])
    v = np.cross(axis, e)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def axis2_of(asm) -> np.ndarray:
    """The assembly's second axes, or perpendiculars of its axes if unset."""
    return perpendicular(asm.axis) if asm.axis2 is None else asm.axis2


def mix_joint_types(asm: Assembly, seed: int, probs=(0.25, 0.25, 0.25, 0.25)) -> Assembly:
    """The assembly with each joint's type redrawn (ball, hinge, universal,
    prismatic with the given probabilities), axes uniform on the sphere and
    second axes uniform on the circle orthogonal to them; anchors unchanged."""
    rng = np.random.default_rng(seed)
    out = asm.copy()
    m = out.m
    out.jtype = rng.choice(4, size=m, p=np.asarray(probs, float) / np.sum(probs)).astype(np.uint8)
    out.axis = _unit_sphere(rng, m)
    u = perpendicular(out.axis)
    w = np.cross(out.axis, u)
    phi = rng.uniform(0.0, 2.0 * np.pi, m)[:, None]
    out.axis2 = np.cos(phi) * u + np.sin(phi) * w
    return out


def concat(parts, name="batch", h=1e-2, steps=100) -> Assembly:
    """One assembly holding independent sub-assemblies (indices shifted)."""
    off = 0
    cols = {k: [] for k in ("dims", "density", "k_orth", "pinned", "q0", "qd0", "jtype",
                             "ja", "jb", "pa", "pb", "axis", "cp_len", "axis2")}
    sizes = []
    for p in parts:
        cols["axis2"].append(axis2_of(p))
        for k in ("dims", "density", "k_orth", "pinned", "q0", "qd0", "jtype", "pa", "pb",
                  "axis", "cp_len"):
            cols[k].append(getattr(p, k))
        cols["ja"].append(np.where(p.ja >= 0, p.ja + off, -1).astype(np.int32))
        cols["jb"].append(np.where(p.jb >= 0, p.jb + off, -1).astype(np.int32))
        sizes.append(p.n)
        off += p.n
    cat = {k: np.concatenate(v) for k, v in cols.items()}
    return Assembly(name=name, h=h, steps=steps, meta=dict(kind="batch", sizes=sizes), **cat)


def batch(count: int = 4096, seed: int = 0, lo: int = 16, hi: int = 4096,
          chain_frac: float = 0.6, h: float = 1e-2, steps: int = 100,
          spacing: float = 10.0) -> Assembly:
    """`count` independent assemblies, sizes round(exp(U(ln lo, ln hi))); each a
    chain (probability chain_frac, chain boxes, ball/hinge 50/50) or a random
    tree (window 64, ball/hinge 50/50); body 0 of each pinned.  Assemblies are
    placed `spacing` metres apart in y."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(int)
    kinds = rng.random(count) < chain_frac
    subseeds = rng.integers(0, 2**31 - 1, size=count)
    parts = []
    for i in range(count):
        org = (0.0, spacing * i, 0.0)
        if kinds[i]:
            parts.append(chain(int(sizes[i]), seed=int(subseeds[i]), hinge_frac=0.5,
                               h=h, steps=steps, origin=org))
        else:
            parts.append(tree(int(sizes[i]), seed=int(subseeds[i]), hinge_frac=0.5,
                              h=h, steps=steps, origin=org))
    a = concat(parts, name=f"batch{count}", h=h, steps=steps)
    a.meta.update(seed=seed, chain=kinds.tolist())
    return a


def lattice(k: int, seed: int = 0, sigma: float = 1e-2, pitch: float = 0.2,
            plate=(0.2, 0.2, 0.05), density: float = 1000.0, k_orth: float = 1e8,
            h: float = 1e-2, steps: int = 100) -> Assembly:
    """k x k plates at `pitch` in the xy plane, z sag N(0, sigma^2); ball joints
    to the 4-neighbours at the midpoint of the two facing edge midpoints; row
    j = 0 pinned; joints between two pinned plates dropped."""
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    idx = (jj * k + ii).ravel()            # body index = j * k + i
    n = k * k
    centres = np.zeros((n, 3))
    centres[idx, 0] = ii.ravel() * pitch
    centres[idx, 1] = jj.ravel() * pitch
    centres[:, 2] = rng.normal(0.0, sigma, size=n)
    pinned = np.zeros(n, np.uint8)
    pinned[:k] = 1                          # row j = 0
    A, B, NA, NB = [], [], [], []
    hx = np.array([0.5 * plate[0], 0.0, 0.0])
    hy = np.array([0.0, 0.5 * plate[1], 0.0])
    for j in range(k):
        for i in range(k):
            b = j * k + i
            if i + 1 < k:
                A.append(b); B.append(b + 1); NA.append(hx); NB.append(-hx)
            if j + 1 < k:
                A.append(b); B.append(b + k); NA.append(hy); NB.append(-hy)
    A = np.asarray(A, np.int32); B = np.asarray(B, np.int32)
    keep = ~((pinned[A] == 1) & (pinned[B] == 1))
    A, B = A[keep], B[keep]
    NA = np.asarray(NA)[keep]; NB = np.asarray(NB)[keep]
    m = A.shape[0]
    jt, ja, jb, pa, pb, ax, ell = _joint_arrays(m)
    ja[:] = A
    jb[:] = B
    pa[:], pb[:] = _midpoint_anchor(centres[A], centres[B], NA, NB)
    return Assembly(
        name=f"lattice{k}", dims=np.tile(np.asarray(plate, float), (n, 1)),
        density=np.full(n, density), k_orth=np.full(n, k_orth), pinned=pinned,
        q0=_identity_q(centres), qd0=np.zeros((n, 12)), jtype=jt, ja=ja, jb=jb,
        pa=pa, pb=pb, axis=ax, cp_len=ell, h=h, steps=steps,
        meta=dict(kind="lattice", seed=seed, k=k))


def rgg(n: int, seed: int = 0, box: Optional[float] = None, radius: float = 1.5,
        knn: int = 4, pin_frac: float = 0.01, cube: float = 0.2, density: float = 1000.0,
        k_orth: float = 1e8, h: float = 1e-2, steps: int = 100) -> Assembly:
    """n cubes at uniform points of a box of side `box` (default keeps the
    density of 100,000 bodies in a 50 m cube); ball joints between each body and
    its <= knn nearest neighbours within `radius` (undirected union), anchored
    at the midpoint of the centres; round(pin_frac * n) bodies pinned."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    if box is None:
        box = 50.0 * (n / 100000.0) ** (1.0 / 3.0)
    centres = rng.uniform(0.0, box, size=(n, 3))
    tree_ = cKDTree(centres)
    dist, nbr = tree_.query(centres, k=knn + 1, distance_upper_bound=radius)
    pairs = set()
    for i in range(n):
        for d, j in zip(dist[i, 1:], nbr[i, 1:]):
            if np.isfinite(d) and j < n and j != i:
                pairs.add((min(i, int(j)), max(i, int(j))))
    pairs = sorted(pairs)
    pinned = np.zeros(n, np.uint8)
    npin = int(round(pin_frac * n))
    if npin:
        pinned[rng.choice(n, size=npin, replace=False)] = 1
    pairs = [p for p in pairs if not (pinned[p[0]] and pinned[p[1]])]
    m = len(pairs)
    jt, ja, jb, pa, pb, ax, ell = _joint_arrays(m)
    if m:
        P = np.asarray(pairs, np.int32)
        ja[:] = P[:, 0]
        jb[:] = P[:, 1]
        mid = 0.5 * (centres[P[:, 0]] + centres[P[:, 1]])
        pa[:] = mid - centres[P[:, 0]]
        pb[:] = mid - centres[P[:, 1]]
    return Assembly(
        name=f"rgg{n}", dims=np.full((n, 3), cube), density=np.full(n, density),
        k_orth=np.full(n, k_orth), pinned=pinned, q0=_identity_q(centres),
        qd0=np.zeros((n, 12)), jtype=jt, ja=ja, jb=jb, pa=pa, pb=pb, axis=ax,
        cp_len=ell, h=h, steps=steps, meta=dict(kind="rgg", seed=seed, box=box))


def free_body(dims=(0.1, 0.1, 0.1), density=1000.0, k_orth=1e8, A=None, t=(0.0, 0.0, 0.0),
              qd=None, h=1e-2) -> Assembly:
    """A single unjointed box (for the single-body pins)."""
    q = _identity_q(np.asarray([t], float))
    if A is not None:
        q[0, 0:9] = np.asarray(A, float).T.reshape(9)   # column-stacked
    qd0 = np.zeros((1, 12)) if qd is None else np.asarray(qd, float).reshape(1, 12)
    jt, ja, jb, pa, pb, ax, ell = _joint_arrays(0)
    return Assembly(name="free", dims=np.asarray([dims], float), density=np.array([density]),
                    k_orth=np.array([k_orth]), pinned=np.zeros(1, np.uint8), q0=q, qd0=qd0,
                    jtype=jt, ja=ja, jb=jb, pa=pa, pb=pb, axis=ax, cp_len=ell, h=h,
                    meta=dict(kind="free"))


def spinning_boxes(n: int, seed: int = 0, dim_range=(0.05, 0.5), density: float = 1000.0,
                   k_orth: float = 1e8, omega: float = 5.0, speed: float = 1.0, h: float = 1e-2,
                   steps: int = 100) -> Assembly:
    """n unjointed boxes on a grid (1 m pitch), each turned to a uniformly
    random orientation and moving rigidly: angular velocity N(0, omega^2) per
    axis, linear velocity N(0, speed^2) per axis (the rigid-body scenes of the
    single-body comparison, Sec. 6.1, as a batch)."""
    rng = np.random.default_rng(seed)
    dims = rng.uniform(dim_range[0], dim_range[1], size=(n, 3))
    side = int(math.ceil(n ** (1.0 / 3.0)))
    idx = np.arange(n)
    centres = np.stack([idx % side, (idx // side) % side, idx // (side * side)], axis=1).astype(float)
    # uniform rotations from unit quaternions
    qu = rng.normal(size=(n, 4))
    qu /= np.linalg.norm(qu, axis=1, keepdims=True)
    w, x, y, z = qu.T
    R = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                  np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                  np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)],
                 axis=1)
    om = rng.normal(0.0, omega, size=(n, 3))
    v = rng.normal(0.0, speed, size=(n, 3))
    q0 = np.zeros((n, 12))
    qd0 = np.zeros((n, 12))
    for c in range(3):
        q0[:, 3 * c:3 * c + 3] = R[:, :, c]
        qd0[:, 3 * c:3 * c + 3] = np.cross(om, R[:, :, c])
    q0[:, 9:] = centres
    qd0[:, 9:] = v
    jt, ja, jb, pa, pb, ax, ell = _joint_arrays(0)
    return Assembly(name=f"boxes{n}", dims=dims, density=np.full(n, density),
                    k_orth=np.full(n, k_orth), pinned=np.zeros(n, np.uint8), q0=q0, qd0=qd0,
                    jtype=jt, ja=ja, jb=jb, pa=pa, pb=pb, axis=ax, cp_len=ell, h=h, steps=steps,
                    meta=dict(kind="boxes", seed=seed))


# The configurations the benchmark and tests run (sizes and settings of the
# paper-shaped workloads; `small` variants finish on the CPU oracle in seconds).
def config(name: str, seed: int = 0) -> Assembly:
    if name == "chain64":
        return chain(64, seed=seed, steps=200)
    if name == "chain1m":
        return chain(1 << 20, seed=seed, steps=100)
    if name == "tree256k":
        return tree(1 << 18, seed=seed, steps=100)
    if name == "batch4096":
        return batch(4096, seed=seed, steps=100)
    if name == "lattice512":
        return lattice(512, seed=seed, steps=100)
    if name == "rgg100k":
        return rgg(100000, seed=seed, steps=100)
    if name == "boxes1m":
        return spinning_boxes(1 << 20, seed=seed, steps=100)
    if name == "hchain1m":  # the C1 chain at 1M links, ball and hinge joints 50/50
        return chain(1 << 20, seed=seed, hinge_frac=0.5, steps=100)
    raise KeyError(name)
