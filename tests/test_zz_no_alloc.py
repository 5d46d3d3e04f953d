"""mabd_residual_noalloc, the residual call for callers that cannot
allocate (partial sums in the library's fixed device array), against
mabd_residual through the C ABI: two calls in a row, the second on a smaller
assembly, bit for bit; and the host-side refusal of an assembly beyond the
fixed array's size."""
import ctypes

import numpy as np
import pytest

import mabd_inputs as mi
from gpu_util import say

pytestmark = pytest.mark.gpu

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None


def noalloc(ctx):
    import torch

    import paper_2603_08079_amd as pk

    out = torch.full((5,), -7.0, dtype=torch.float64, device="cuda")
    st = pk.lib().mabd_residual_noalloc(ctx.h, ctypes.c_void_p(out.data_ptr()))
    torch.cuda.synchronize()
    return st, out.cpu().numpy()


def test_noalloc_residual_matches_the_allocating_call():
    import paper_2603_08079_amd as pk

    big = mi.concat([mi.chain(20000, seed=81), mi.tree(3000, seed=82, origin=(0.0, 40.0, 0.0))])
    big.qd0[1:] = np.random.default_rng(81).normal(0, 0.05, (big.n - 1, 12))
    small = mi.tree(300, seed=83)
    small.qd0[1:] = np.random.default_rng(83).normal(0, 0.05, (small.n - 1, 12))
    cb, cs = pk.Context(big), pk.Context(small)
    cb.step(big.h, 2)
    cs.step(small.h, 1)
    for ctx, name in ((cb, "chain 20000 + tree 3000"), (cs, "tree 300")):
        st, v = noalloc(ctx)
        assert st == pk.OK, pk.lib().mabd_last_error(ctx.h)
        r = ctx.residual()
        ref = np.array([r[k] for k in ("rho_p", "rho_d", "kkt", "c_ball", "c_hinge")])
        say(name, "noalloc", v, "residual", ref)
        assert np.array_equal(v, ref), (v, ref)
        assert 0.0 <= v[2] < 1e-10


def test_noalloc_refuses_beyond_its_records():
    import paper_2603_08079_amd as pk

    # 65,537 chain tiles of 60 rows: one record more than the fixed array holds
    n = 60 * 65536 + 62
    asm = mi.chain(n, seed=84)
    ctx = pk.Context(asm, autotune=0)
    st, v = noalloc(ctx)
    assert st == pk.ERR_INVALID_ARG
    assert "fixed scratch" in pk.lib().mabd_last_error(ctx.h).decode()
    assert np.all(v == -7.0)  # nothing was queued
