"""FP64 CPU oracle for the M-ABD per-step solve (arXiv 2603.08079).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It never imports
the GPU package and the GPU package never imports it.

The C source (``mabd_oracle.c``) holds the arithmetic; this module marshals
numpy arrays into it and adds one step that is a library call: solving the
assembled sparse dual system with SciPy's SuperLU for graphs too large for the
dense Cholesky path (Sec. 5.1 allows "any linear solver").

Parity status per function (pins live in tests/test_oracle_pins.py and
tests/test_oracle_verifier.py):
  * single-body step, free flight .......... pinned (closed-form implicit Euler)
  * co-rotated elastic step ................ pinned (closed-form linear oscillator,
                                              rotation equivariance)
  * ball joints, chain/tree/dense solvers .. pinned (dense KKT LU, exact constraint
                                              residual, pendulum convergence)
  * hinge joints ........................... pinned (finite differences of the
                                              constraint at rest and, away from
                                              rest, along rigid motions; hinge
                                              pendulum; rows of the second point
                                              normal to the axis); the
                                              A-linearised rotation term along
                                              stretch directions is a reading of
                                              Eq. r_gradient
  * PCG .................................... pinned against the dense solve
  * verifier (residual) .................... pinned (closed-form rho_d of scaled
                                              multipliers, brute-force KKT
                                              residuals, anchor distances)
  * twists and joint wrenches .............. pinned (rigid spin closed form,
                                              wrench round trip through G(A)^T,
                                              action and reaction of internal
                                              joints, a hanging body carrying
                                              its weight)

tests/test_oracle_mutants.py plants mistakes in copies of the C source and
checks that these pins catch them.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmabd_oracle.so")

AUTO, CHAIN, TREE, DENSE, PCG = 0, 1, 2, 3, 4
RHO_P, RHO_D, KKT, CBALL, CHINGE, ITERS, SOLVER = range(7)
NDIAG = 8


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


class _Sys(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("dims", ctypes.c_void_p), ("density", ctypes.c_void_p), ("k_orth", ctypes.c_void_p),
        ("poisson", ctypes.c_void_p), ("pinned", ctypes.c_void_p), ("q0", ctypes.c_void_p),
        ("m", ctypes.c_int32),
        ("jtype", ctypes.c_void_p), ("ja", ctypes.c_void_p), ("jb", ctypes.c_void_p),
        ("pa", ctypes.c_void_p), ("pb", ctypes.c_void_p), ("axis", ctypes.c_void_p),
        ("cp_len", ctypes.c_void_p),
        ("gravity", ctypes.c_double * 3),
        ("material", ctypes.c_int32), ("hinge_grad", ctypes.c_int32),
        ("newton_iters", ctypes.c_int32),
        ("wrench", ctypes.c_void_p),
        ("axis2", ctypes.c_void_p),
        ("body_solve", ctypes.c_int32),
    ]


_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, FP64, one thread)."""
    import subprocess

    src = os.path.join(_HERE, "mabd_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-march=x86-64-v3", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_native(path: str, openmp: bool) -> str:
    """Compile a copy of the oracle for the machine it runs on (-O3
    -march=native, with or without OpenMP over the per-body phases) at `path`;
    the arithmetic is the same source.  Used for the CPU baseline timing."""
    import subprocess

    src = os.path.join(_HERE, "mabd_oracle.c")
    cmd = ["gcc", "-O3", "-march=native", "-std=c99", "-fPIC", "-shared"]
    if openmp:
        cmd.append("-fopenmp")
    subprocess.check_call(cmd + ["-o", path, src, "-lm"])
    return path


def load(path: str):
    """Load an oracle library built by build_native (CPU baseline only)."""
    return _declare(ctypes.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _declare(L):
    """Argument and result types of the exported oracle calls."""
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.ora_polar.argtypes = [P, P]; L.ora_polar.restype = I32
    L.ora_rows.argtypes = [P]; L.ora_rows.restype = I32
    L.ora_classify.argtypes = [P]; L.ora_classify.restype = I32
    L.ora_step.argtypes = [P, D, P, P, I32, D, I32, P, P]; L.ora_step.restype = I32
    L.ora_body_terms.argtypes = [P, D, P, P, I32, P, P, P]; L.ora_body_terms.restype = I32
    L.ora_joint_terms.argtypes = [P, P, I32, P, P, P]; L.ora_joint_terms.restype = I32
    L.ora_dual_coo.argtypes = [P, D, P, P, I64, P, P, P, P]; L.ora_dual_coo.restype = I64
    L.ora_finish.argtypes = [P, D, P, P, P, P, P, P]; L.ora_finish.restype = I32
    L.ora_residual.argtypes = [P, D, P, P, P, P, P, P]; L.ora_residual.restype = I32
    L.ora_twists.argtypes = [P, P, P, P]; L.ora_twists.restype = I32
    L.ora_joint_wrenches.argtypes = [P, P, P, P]; L.ora_joint_wrenches.restype = I32
    return L


def _p(a):
    return None if a is None else a.ctypes.data


class System:
    """Holds contiguous copies of an assembly's arrays and the C struct."""

    def __init__(self, asm, material: Optional[int] = None, hinge_grad: int = 0,
                 newton_iters: int = 1, gravity=None, wrench=None, L=None, body_solve: int = 0):
        # L: an oracle library loaded with load() (the same source built for
        # the host, for the CPU baseline timing); default: the test build
        self.L = lib() if L is None else L
        c = np.ascontiguousarray
        self.n, self.m = asm.n, asm.m
        self.dims = c(asm.dims, np.float64)
        self.density = c(asm.density, np.float64)
        self.k_orth = c(asm.k_orth, np.float64)
        self.poisson = None if asm.poisson is None else c(asm.poisson, np.float64)
        self.pinned = c(asm.pinned, np.uint8)
        self.q0 = c(asm.q0, np.float64)
        self.jtype = c(asm.jtype, np.uint8)
        self.ja = c(asm.ja, np.int32)
        self.jb = c(asm.jb, np.int32)
        self.pa = c(asm.pa, np.float64)
        self.pb = c(asm.pb, np.float64)
        self.axis = c(asm.axis, np.float64)
        self.cp_len = c(asm.cp_len, np.float64)
        a2 = getattr(asm, "axis2", None)
        self.axis2 = None if a2 is None else c(a2, np.float64)
        # external wrench per body [tau; f] (world frame, about the COM), or None
        self.wrench = None if wrench is None else c(np.asarray(wrench, np.float64).reshape(self.n, 6))
        s = _Sys()
        s.n, s.m = self.n, self.m
        for f in ("dims", "density", "k_orth", "poisson", "pinned", "q0", "jtype", "ja", "jb",
                  "pa", "pb", "axis", "cp_len", "wrench", "axis2"):
            setattr(s, f, _p(getattr(self, f)))
        g = asm.gravity if gravity is None else gravity
        s.gravity[0], s.gravity[1], s.gravity[2] = g
        s.material = asm.material if material is None else material
        s.hinge_grad = hinge_grad
        s.newton_iters = newton_iters
        s.body_solve = body_solve
        self.s = s
        self.rows = self.L.ora_rows(ctypes.byref(s))

    @property
    def ref(self):
        return ctypes.byref(self.s)

    def classify(self) -> int:
        return self.L.ora_classify(self.ref)

    def step(self, h, q, qd, solver=AUTO, tol=1e-10, max_iters=100000):
        """One time step.  Returns (q1, qd1, lam, diag)."""
        q1 = np.array(q, np.float64, order="C", copy=True)
        qd1 = np.array(qd, np.float64, order="C", copy=True)
        lam = np.zeros(max(self.rows, 1))
        diag = np.zeros(NDIAG)
        st = self.L.ora_step(self.ref, h, _p(q1), _p(qd1), solver, tol, max_iters, _p(lam),
                            _p(diag))
        if st != 0:
            raise OracleError(st, "step")
        return q1, qd1, lam[: self.rows], diag

    def body_terms(self, h, q, qd, i):
        H = np.zeros((12, 12)); f = np.zeros(12); R = np.zeros(9)
        q = np.ascontiguousarray(q, np.float64); qd = np.ascontiguousarray(qd, np.float64)
        st = self.L.ora_body_terms(self.ref, h, _p(q), _p(qd), i, _p(H), _p(f), _p(R))
        if st != 0:
            raise OracleError(st, "body_terms")
        return H, f, R

    def joint_terms(self, q, k):
        C = np.zeros(5); Ga = np.zeros((5, 12)); Gb = np.zeros((5, 12))
        q = np.ascontiguousarray(q, np.float64)
        st = self.L.ora_joint_terms(self.ref, _p(q), k, _p(C), _p(Ga), _p(Gb))
        if st != 0:
            raise OracleError(st, "joint_terms")
        r = (3, 5, 4, 5)[int(self.jtype[k])]  # rows per joint type
        return C[:r], Ga[:r], Gb[:r]

    def dual(self, h, q, qd):
        """Sparse dual matrix S (scipy CSR) and right-hand side r."""
        import scipy.sparse as sp

        q = np.ascontiguousarray(q, np.float64); qd = np.ascontiguousarray(qd, np.float64)
        nnz = self.L.ora_dual_coo(self.ref, h, _p(q), _p(qd), 0, None, None, None, None)
        if nnz < 0:
            raise OracleError(int(nnz), "dual_coo")
        I = np.zeros(max(nnz, 1), np.int64); J = np.zeros(max(nnz, 1), np.int64)
        V = np.zeros(max(nnz, 1)); r = np.zeros(max(self.rows, 1))
        self.L.ora_dual_coo(self.ref, h, _p(q), _p(qd), nnz, _p(I), _p(J), _p(V), _p(r))
        S = sp.coo_matrix((V[:nnz], (I[:nnz], J[:nnz])), shape=(self.rows, self.rows)).tocsr()
        return S, r[: self.rows]

    def finish(self, h, q, qd, lam):
        """Back-projection and diagnostics for given multipliers (one Newton iteration)."""
        q = np.ascontiguousarray(q, np.float64); qd = np.ascontiguousarray(qd, np.float64)
        lam = np.ascontiguousarray(lam, np.float64)
        q1 = np.zeros_like(q); qd1 = np.zeros_like(qd); diag = np.zeros(NDIAG)
        st = self.L.ora_finish(self.ref, h, _p(q), _p(qd), _p(lam), _p(q1), _p(qd1), _p(diag))
        if st != 0:
            raise OracleError(st, "finish")
        return q1, qd1, diag

    def residual(self, h, q, qd, dq, lam, q_new=None):
        """Verifier of a step computed elsewhere: the KKT residuals (rho_p,
        rho_d, max of both) of the increment dq and multipliers lam for the
        state (q, qd), and the post-step constraint values at q_new (q + dq if
        None).  Nothing is solved.  Returns the diag vector."""
        c = np.ascontiguousarray
        q = c(q, np.float64); qd = c(qd, np.float64); dq = c(dq, np.float64)
        lam = c(lam, np.float64)
        qn = None if q_new is None else c(q_new, np.float64)
        diag = np.zeros(NDIAG)
        st = self.L.ora_residual(self.ref, h, _p(q), _p(qd), _p(dq), _p(lam), _p(qn), _p(diag))
        if st != 0:
            raise OracleError(st, "residual")
        return diag

    def twists(self, q, qd):
        """Spatial twist [omega; v] of every body (n x 6)."""
        c = np.ascontiguousarray
        q = c(q, np.float64); qd = c(qd, np.float64)
        V = np.zeros((self.n, 6))
        st = self.L.ora_twists(self.ref, _p(q), _p(qd), _p(V))
        if st != 0:
            raise OracleError(st, "twists")
        return V

    def joint_wrenches(self, q, lam):
        """Spatial wrench [tau; f] (about the COM) of the joint forces of a
        step from q with multipliers lam, on every body (n x 6)."""
        c = np.ascontiguousarray
        q = c(q, np.float64); lam = c(lam, np.float64)
        W = np.zeros((self.n, 6))
        st = self.L.ora_joint_wrenches(self.ref, _p(q), _p(lam), _p(W))
        if st != 0:
            raise OracleError(st, "joint_wrenches")
        return W

    def step_sparse(self, h, q, qd):
        """One step with the dual solved by SciPy SuperLU (graphs at reduced sizes)."""
        import scipy.sparse.linalg as spla

        S, r = self.dual(h, q, qd)
        lam = spla.splu(S.tocsc()).solve(r)
        q1, qd1, diag = self.finish(h, q, qd, lam)
        return q1, qd1, lam, diag


def polar(A):
    """Polar factor of a 3x3 matrix (row-major numpy array) via the oracle."""
    A = np.asarray(A, np.float64)
    Aq = np.ascontiguousarray(A.T.reshape(9))
    Rq = np.zeros(9)
    st = lib().ora_polar(_p(Aq), _p(Rq))
    if st != 0:
        raise OracleError(st, "polar")
    return Rq.reshape(3, 3).T.copy()


def run(asm, steps=None, solver=AUTO, **kw):
    """Integrate `steps` steps from the assembly's initial state."""
    sysm = System(asm, **{k: v for k, v in kw.items() if k in ("material", "hinge_grad",
                                                                "newton_iters", "gravity", "wrench",
                                                                "body_solve")})
    q, qd = asm.q0.copy(), asm.qd0.copy()
    diags = []
    for _ in range(asm.steps if steps is None else steps):
        q, qd, lam, d = sysm.step(asm.h, q, qd, solver=solver,
                                  tol=kw.get("tol", 1e-10), max_iters=kw.get("max_iters", 100000))
        diags.append(d)
    return q, qd, np.asarray(diags)
