"""A plain C99 program as a client of the C ABI (tests/abi_client.c): it
includes only include/mabd.h, links libmabd.so with gcc, and steps an
assembly through mabd_options_default / mabd_create / mabd_step /
mabd_state / mabd_multipliers / mabd_residual / mabd_destroy.  On the CPU the
program must compile without warnings and link against every symbol it
uses; on the GPU its state, multipliers and residual must be bitwise those
of the Python binding on the same input (ball chain on the fused chain path,
a tree of all four joint types on the tree contraction, and free boxes)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import mabd_inputs as mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_08079_amd")
LIB = os.path.join(PKG, "libmabd.so")
SRC = os.path.join(ROOT, "tests", "abi_client.c")


def build_client(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libmabd.so is not built")
    exe = str(tmp_path / "abi_client")
    subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I",
                    os.path.join(ROOT, "include"), "-o", exe, SRC, "-L", PKG, "-lmabd",
                    "-Wl,-rpath," + PKG], check=True, capture_output=True, text=True)
    return exe


def test_client_compiles_and_links(tmp_path):
    exe = build_client(tmp_path)
    # every undefined mabd_ symbol of the program resolves in the library
    und = subprocess.run(["nm", "-u", exe], capture_output=True, text=True, check=True).stdout
    used = sorted({ln.split()[-1].split("@")[0] for ln in und.splitlines() if "mabd_" in ln})
    dyn = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    have = {ln.split()[-1] for ln in dyn.splitlines() if ln.split()}
    assert len(used) >= 8 and set(used) <= have, sorted(set(used) - have)


def assembly():
    c = mi.chain(300, seed=171)
    t = mi.mix_joint_types(mi.tree(500, seed=172, window=8), seed=173)
    t.q0[:, 9:] += np.array([0.0, 30.0, 0.0])
    boxes = mi.concat([mi.free_body(t=(float(i), -20.0, 0.0)) for i in range(40)])
    a = mi.concat([c, t, boxes], h=1e-2, steps=4)
    rng = np.random.default_rng(174)
    a.qd0[:] = rng.normal(0, 0.05, a.qd0.shape)
    a.qd0[a.pinned == 1] = 0.0
    return a


def write_input(path, a, steps):
    with open(path, "wb") as f:
        f.write(np.array([a.n, a.m, steps], np.int32).tobytes())
        f.write(np.array([a.h], np.float64).tobytes())
        for arr, dt in ((a.dims, np.float64), (a.density, np.float64), (a.k_orth, np.float64),
                        (a.pinned, np.uint8), (a.q0, np.float64), (a.qd0, np.float64),
                        (a.jtype, np.uint8), (a.ja, np.int32), (a.jb, np.int32),
                        (a.pa, np.float64), (a.pb, np.float64), (a.axis, np.float64),
                        (a.cp_len, np.float64), (mi.axis2_of(a), np.float64)):
            f.write(np.ascontiguousarray(arr, dt).tobytes())


def read_output(path, n):
    raw = open(path, "rb").read()
    st, rows = np.frombuffer(raw[:8], np.int32)
    d = np.frombuffer(raw[8:], np.float64)
    q, qd = d[:12 * n].reshape(n, 12), d[12 * n:24 * n].reshape(n, 12)
    lam, res = d[24 * n:24 * n + rows], d[24 * n + rows:]
    assert res.shape == (5,)
    return int(st), q, qd, lam, res


@pytest.mark.gpu
def test_c_client_matches_the_python_binding(tmp_path):
    import paper_2603_08079_amd as pk

    exe = build_client(tmp_path)
    a = assembly()
    a.axis2 = mi.axis2_of(a)
    steps = 4
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_input(inp, a, steps)
    print("C client: n", a.n, "m", a.m, "steps", steps, flush=True)
    r = subprocess.run(["timeout", "-k", "10", "120", exe, inp, out], capture_output=True,
                       text=True)
    sys.stdout.write(r.stderr)
    assert r.returncode == 0, r.stderr
    st, q, qd, lam, res = read_output(out, a.n)
    assert st == 0

    ctx = pk.Context(a)
    ctx.step(a.h, steps)
    qp, qdp = ctx.state()
    lp = ctx.multipliers()
    rp = ctx.residual()
    stats = ctx.stats()
    ctx.close()
    print("rows", lam.size, "n_chain", stats["n_chain"], "n_tree", stats["n_tree"],
          "residual", res, flush=True)
    assert stats["n_chain"] > 0 and stats["n_tree"] > 0
    assert lam.size == lp.size == a.rows()
    assert np.array_equal(q, qp) and np.array_equal(qd, qdp)
    assert np.array_equal(lam, lp)
    assert np.array_equal(res, np.array([rp[k] for k in ("rho_p", "rho_d", "kkt", "c_ball", "c_hinge")]))
    assert np.all(np.isfinite(q)) and np.abs(q - a.q0).max() > 0
