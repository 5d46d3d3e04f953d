"""Python binding of libmabd, the MI355X implementation of the M-ABD per-step
solve (arXiv 2603.08079).  Argument marshalling only: every step of the
solve runs in the library's HIP kernels.  PyTorch supplies device memory and
streams where the caller wants device-side state.

The binding refuses to run without the compiled library: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmabd.so")

OK, ERR_INVALID_ARG, ERR_TOPOLOGY, ERR_DEVICE, ERR_OOM, ERR_NONFINITE, ERR_NOT_CONVERGED, \
    ERR_SINGULAR = 0, -1, -2, -3, -4, -5, -6, -7

EXPORTED = ["mabd_options_default", "mabd_create", "mabd_step", "mabd_state", "mabd_state_device",
            "mabd_set_state", "mabd_set_wrenches", "mabd_multipliers", "mabd_rows", "mabd_residual", "mabd_residual_noalloc",
            "mabd_twists", "mabd_joint_wrenches",
            "mabd_stats",
            "mabd_gnn_size",
            "mabd_gnn_init", "mabd_gnn_params", "mabd_gnn_grad", "mabd_gnn_train", "mabd_gnn_predict",
            "mabd_gnn_save", "mabd_gnn_load", "mabd_last_error", "mabd_destroy"]


class MabdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mabd status {status}: {msg}")
        self.status = status


class Bodies(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32),
                ("dims", ctypes.c_void_p), ("density", ctypes.c_void_p),
                ("k_orth", ctypes.c_void_p), ("poisson", ctypes.c_void_p),
                ("pinned", ctypes.c_void_p), ("q0", ctypes.c_void_p), ("qd0", ctypes.c_void_p)]


class Joints(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32),
                ("type", ctypes.c_void_p), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("pa", ctypes.c_void_p), ("pb", ctypes.c_void_p), ("axis", ctypes.c_void_p),
                ("cp_len", ctypes.c_void_p), ("axis2", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("gravity", ctypes.c_double * 3), ("precision", ctypes.c_int32),
                ("kkt_tol", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("hinge_grad", ctypes.c_int32), ("material", ctypes.c_int32),
                ("diagnostics", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("ir_max_sweeps", ctypes.c_int32),
                ("body_solve", ctypes.c_int32), ("path_solver", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
                ("stream", ctypes.c_void_p)]


NPHASES = 10
NEWTON_DIAG = 8


class StepStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int64), ("last_status", ctypes.c_int32),
                ("pcg_iters", ctypes.c_int32), ("rho_p", ctypes.c_double),
                ("rho_d", ctypes.c_double), ("kkt", ctypes.c_double),
                ("c_ball", ctypes.c_double), ("c_hinge", ctypes.c_double),
                ("ir_sweeps", ctypes.c_int32), ("warm_accepted", ctypes.c_int32),
                ("n_chain", ctypes.c_int32), ("n_tree", ctypes.c_int32),
                ("n_graph", ctypes.c_int32), ("n_dyn", ctypes.c_int32),
                ("phase_ms", ctypes.c_double * NPHASES), ("phase_calls", ctypes.c_int64 * NPHASES),
                ("tile_threads", ctypes.c_int32), ("graph_replay", ctypes.c_int32),
                ("tree_rounds", ctypes.c_int32), ("tile_packed", ctypes.c_int32),
                ("ir_stalled", ctypes.c_int32), ("kkt_newton", ctypes.c_double * NEWTON_DIAG),
                ("n_loop", ctypes.c_int32), ("tree_split", ctypes.c_int32),
                ("tree_order", ctypes.c_int32), ("tune_source", ctypes.c_int32),
                ("n_path", ctypes.c_int32), ("path_levels", ctypes.c_int32)]

    PHASES = ("chain_reduce", "chain_global", "chain_apply", "body", "joint", "tree", "apply",
              "pcg", "chain_resid", "chain_finish")

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        d["phase_calls"] = list(self.phase_calls)
        d["kkt_newton"] = list(self.kkt_newton)
        return d


_lib = None


def lib():
    """Load libmabd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2603_08079_amd/build.py "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.mabd_options_default.argtypes = [P]; L.mabd_options_default.restype = None
        L.mabd_create.argtypes = [P, P, P, P]; L.mabd_create.restype = I32
        L.mabd_step.argtypes = [P, D, I32]; L.mabd_step.restype = I32
        L.mabd_state.argtypes = [P, P, P]; L.mabd_state.restype = I32
        L.mabd_state_device.argtypes = [P, P, P]; L.mabd_state_device.restype = I32
        L.mabd_set_state.argtypes = [P, P, P]; L.mabd_set_state.restype = I32
        L.mabd_set_wrenches.argtypes = [P, P]; L.mabd_set_wrenches.restype = I32
        L.mabd_multipliers.argtypes = [P, P]; L.mabd_multipliers.restype = I32
        L.mabd_rows.argtypes = [P]; L.mabd_rows.restype = I64
        L.mabd_stats.argtypes = [P, P]; L.mabd_stats.restype = I32
        L.mabd_residual.argtypes = [P, P]; L.mabd_residual.restype = I32
        L.mabd_residual_noalloc.argtypes = [P, P]; L.mabd_residual_noalloc.restype = I32
        L.mabd_twists.argtypes = [P, P]; L.mabd_twists.restype = I32
        L.mabd_joint_wrenches.argtypes = [P, P]; L.mabd_joint_wrenches.restype = I32
        L.mabd_gnn_load.argtypes = [P, ctypes.c_char_p]; L.mabd_gnn_load.restype = I32
        L.mabd_gnn_save.argtypes = [P, ctypes.c_char_p]; L.mabd_gnn_save.restype = I32
        L.mabd_gnn_size.argtypes = []; L.mabd_gnn_size.restype = I32
        L.mabd_gnn_init.argtypes = [P, ctypes.c_uint64]; L.mabd_gnn_init.restype = I32
        L.mabd_gnn_params.argtypes = [P, P, P, I32]; L.mabd_gnn_params.restype = I32
        L.mabd_gnn_grad.argtypes = [P, D, P, P]; L.mabd_gnn_grad.restype = I32
        L.mabd_gnn_train.argtypes = [P, D, I32, ctypes.c_float, P, P]; L.mabd_gnn_train.restype = I32
        L.mabd_gnn_predict.argtypes = [P, D, P]; L.mabd_gnn_predict.restype = I32
        L.mabd_last_error.argtypes = [P]; L.mabd_last_error.restype = ctypes.c_char_p
        L.mabd_destroy.argtypes = [P]; L.mabd_destroy.restype = None
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    lib().mabd_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "gravity":
            o.gravity[0], o.gravity[1], o.gravity[2] = v
        elif k == "tune_cache":
            o.tune_cache = None if v is None else os.fsencode(v)
        else:
            setattr(o, k, v)
    return o


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class Context:
    """One assembly on the GPU.  Wraps mabd_create / mabd_step / mabd_state."""

    def __init__(self, asm, stream=None, **opts):
        L = lib()
        self._keep = []
        f64, u8, i32 = np.float64, np.uint8, np.int32
        arrs = dict(dims=_c(asm.dims, f64), density=_c(asm.density, f64),
                    k_orth=_c(asm.k_orth, f64), poisson=_c(asm.poisson, f64),
                    pinned=_c(asm.pinned, u8), q0=_c(asm.q0, f64), qd0=_c(asm.qd0, f64),
                    type=_c(asm.jtype, u8), a=_c(asm.ja, i32), b=_c(asm.jb, i32),
                    pa=_c(asm.pa, f64), pb=_c(asm.pb, f64), axis=_c(asm.axis, f64),
                    cp_len=_c(asm.cp_len, f64), axis2=_c(getattr(asm, "axis2", None), f64))
        self._keep.append(arrs)
        p = lambda x: None if x is None else x.ctypes.data
        B = Bodies(asm.n, p(arrs["dims"]), p(arrs["density"]), p(arrs["k_orth"]),
                   p(arrs["poisson"]), p(arrs["pinned"]), p(arrs["q0"]), p(arrs["qd0"]))
        J = Joints(asm.m, p(arrs["type"]), p(arrs["a"]), p(arrs["b"]), p(arrs["pa"]),
                   p(arrs["pb"]), p(arrs["axis"]), p(arrs["cp_len"]), p(arrs["axis2"]))
        opts.setdefault("gravity", tuple(asm.gravity))
        opts.setdefault("material", asm.material)
        if stream is not None:
            opts["stream"] = stream
        O = default_options(**opts)
        h = ctypes.c_void_p()
        st = L.mabd_create(ctypes.byref(B), ctypes.byref(J), ctypes.byref(O), ctypes.byref(h))
        if st != OK:
            raise MabdError(st, L.mabd_last_error(None).decode())
        self.h = h
        self.n, self.m = asm.n, asm.m
        self.rows = int(L.mabd_rows(h))

    def _check(self, st):
        if st != OK:
            raise MabdError(st, lib().mabd_last_error(self.h).decode())

    def step(self, h: float, n: int = 1):
        self._check(lib().mabd_step(self.h, float(h), int(n)))

    def state(self):
        q = np.zeros((self.n, 12)); qd = np.zeros((self.n, 12))
        self._check(lib().mabd_state(self.h, q.ctypes.data, qd.ctypes.data))
        return q, qd

    def state_device(self, q_dev, qd_dev):
        """Write the state into device tensors (n x 12 float64, contiguous)."""
        for t in (q_dev, qd_dev):
            if t is not None and (not t.is_cuda or t.dtype.itemsize != 8 or not t.is_contiguous()
                                  or t.numel() != 12 * self.n):
                raise ValueError("state_device needs contiguous float64 device tensors of n*12")
        self._check(lib().mabd_state_device(self.h, None if q_dev is None else q_dev.data_ptr(),
                                            None if qd_dev is None else qd_dev.data_ptr()))

    def set_state(self, q, qd):
        q = np.ascontiguousarray(q, np.float64); qd = np.ascontiguousarray(qd, np.float64)
        self._check(lib().mabd_set_state(self.h, q.ctypes.data, qd.ctypes.data))

    def set_wrenches(self, w):
        """External wrenches [tau; f] per body (n x 6, world frame, about the
        COM), applied from the next step on; None removes them."""
        if w is None:
            self._check(lib().mabd_set_wrenches(self.h, None))
            return
        w = np.ascontiguousarray(w, np.float64).reshape(-1, 6)
        if w.shape[0] != self.n:
            raise ValueError(f"wrench array has {w.shape[0]} rows, the assembly {self.n} bodies")
        self._check(lib().mabd_set_wrenches(self.h, w.ctypes.data))

    def multipliers(self):
        lam = np.zeros(max(self.rows, 1))
        self._check(lib().mabd_multipliers(self.h, lam.ctypes.data))
        return lam[: self.rows]

    def residual(self) -> dict:
        """FP64 KKT residual of the last completed step, evaluated on the device."""
        out = np.zeros(5)
        self._check(lib().mabd_residual(self.h, out.ctypes.data))
        return dict(zip(("rho_p", "rho_d", "kkt", "c_ball", "c_hinge"), out.tolist()))

    def residual_noalloc(self, out_dev):
        """The same five values written into a device tensor of 5 float64
        (contiguous) on the context's stream, with the library's fixed
        scratch; returns without waiting."""
        if not out_dev.is_cuda or out_dev.dtype.itemsize != 8 or out_dev.numel() < 5 \
                or not out_dev.is_contiguous():
            raise ValueError("residual_noalloc needs a contiguous float64 device tensor of 5")
        self._check(lib().mabd_residual_noalloc(self.h, out_dev.data_ptr()))

    def twists(self) -> np.ndarray:
        """Spatial twist [omega; v] of every body at the current state (n x 6)."""
        V = np.zeros((self.n, 6))
        self._check(lib().mabd_twists(self.h, V.ctypes.data))
        return V

    def joint_wrenches(self) -> np.ndarray:
        """Spatial wrench [tau; f] of the last step's joint forces on every
        body, about its centre of mass (n x 6)."""
        W = np.zeros((self.n, 6))
        self._check(lib().mabd_joint_wrenches(self.h, W.ctypes.data))
        return W

    def stats(self) -> dict:
        s = StepStats()
        self._check(lib().mabd_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    # ---- learned warm start (warm_start = 2)
    def gnn_init(self, seed: int = 0):
        self._check(lib().mabd_gnn_init(self.h, ctypes.c_uint64(seed)))

    def gnn_params(self, set_to=None) -> np.ndarray:
        n = lib().mabd_gnn_size()
        out = np.zeros(n, np.float32)
        src = None
        if set_to is not None:
            src = np.ascontiguousarray(set_to, np.float32)
            assert src.shape == (n,)
        self._check(lib().mabd_gnn_params(self.h, out.ctypes.data,
                                          None if src is None else src.ctypes.data, n))
        return out

    def gnn_grad(self, h: float):
        g = np.zeros(lib().mabd_gnn_size(), np.float32)
        loss = ctypes.c_double()
        self._check(lib().mabd_gnn_grad(self.h, h, g.ctypes.data, ctypes.byref(loss)))
        return g, loss.value

    def gnn_train(self, h: float, iters: int, lr: float):
        l0, l1 = ctypes.c_double(), ctypes.c_double()
        self._check(lib().mabd_gnn_train(self.h, h, iters, lr, ctypes.byref(l0), ctypes.byref(l1)))
        return l0.value, l1.value

    def gnn_predict(self, h: float) -> np.ndarray:
        lam = np.zeros((max(self.m, 1), 3))
        self._check(lib().mabd_gnn_predict(self.h, h, lam.ctypes.data))
        return lam[: self.m]

    def gnn_save(self, path: str):
        self._check(lib().mabd_gnn_save(self.h, path.encode()))

    def gnn_load(self, path: str):
        self._check(lib().mabd_gnn_load(self.h, path.encode()))

    def close(self):
        if getattr(self, "h", None):
            lib().mabd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
