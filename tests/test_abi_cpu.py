"""C-ABI checks that need no GPU: the library loads, exports every function
include/mabd.h declares, and rejects bad input before touching the device."""
import os
import re

import numpy as np
import pytest

import mabd_inputs as mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mabd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mabd_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import ctypes

    import paper_2603_08079_amd as pk

    L = pk.lib()
    names = header_functions()
    assert "mabd_create" in names and "mabd_step" in names and "mabd_state" in names
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(pk.EXPORTED)


def test_options_default():
    import paper_2603_08079_amd as pk

    o = pk.default_options()
    assert tuple(o.gravity) == (0.0, 0.0, -9.8)
    assert o.newton_iters == 1 and o.kkt_tol == 1e-10 and o.material == 0
    assert o.precision == 0 and o.use_graph == 1 and o.autotune == 1 and o.ir_max_sweeps == 4


def _expect(asm, status, **kw):
    import paper_2603_08079_amd as pk

    with pytest.raises(pk.MabdError) as ei:
        pk.Context(asm, **kw)
    assert ei.value.status == status, str(ei.value)
    return str(ei.value)


def test_invalid_inputs_are_rejected_before_device_work():
    import paper_2603_08079_amd as pk

    base = mi.chain(5, seed=0, hinge_frac=1.0)
    a = base.copy(); a.ja[1] = 99
    assert "body index" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.axis[2] = 0.0
    assert "hinge axis" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.cp_len[0] = 0.0
    assert "cp_len" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.q0[2, 0] = -1.0
    assert "det A" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.dims[1, 0] = 0.0
    assert "dims" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.q0[3, 9] = np.nan
    assert "not finite" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.ja[0] = a.jb[0]
    assert "a == b" in _expect(a, pk.ERR_INVALID_ARG)
    a = base.copy(); a.pinned[:] = 1
    assert "no dynamic side" in _expect(a, pk.ERR_INVALID_ARG)
    _expect(base, pk.ERR_INVALID_ARG, newton_iters=0)
    _expect(base, pk.ERR_INVALID_ARG, hinge_grad=1)
    assert "precision" in _expect(base, pk.ERR_INVALID_ARG, precision=2)
    assert "ir_max_sweeps" in _expect(base, pk.ERR_INVALID_ARG, precision=1, ir_max_sweeps=-1)
    u = mi.mix_joint_types(mi.chain(5, seed=1), seed=2, probs=(0, 0, 1, 0))
    a = u.copy(); a.axis2[2] = a.axis[2]
    assert "orthogonal" in _expect(a, pk.ERR_INVALID_ARG)
    a = u.copy(); a.axis2 = None
    assert "axis2" in _expect(a, pk.ERR_INVALID_ARG)
    a = u.copy(); a.jtype[1] = 4
    assert "type" in _expect(a, pk.ERR_INVALID_ARG)


def test_missing_library_fails_loudly():
    """Without libmabd.so the binding raises at the first call: no fallback."""
    import subprocess
    import sys

    code = ("import paper_2603_08079_amd as pk\n"
            "pk.LIB_PATH = '/nonexistent/libmabd.so'\n"
            "pk._lib = None\n"
            "try:\n"
            "    pk.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "no CPU fallback" in r.stdout
