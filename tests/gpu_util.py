"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(x, ref, floor=0.0):
    scale = max(float(np.abs(ref).max()), floor)
    if scale == 0.0:
        return float(np.abs(x - ref).max())
    return float(np.abs(x - ref).max()) / scale


def state_errors(qg, qdg, qo, qdo):
    """Relative state errors: positions/affine entries against the largest
    coordinate, velocities against the largest velocity."""
    return rel_err(qg, qo, 1.0), rel_err(qdg, qdo, 1e-12)
