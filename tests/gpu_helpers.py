"""Shared helpers of the GPU parity tests (conversions and seeded inputs)."""
import sys

import numpy as np

from oracle import g1
from workloads import ints_to_limbs, limbs_to_ints


def log(*a):
    """Progress line naming the case, flushed before the GPU step it precedes."""
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def points_from_host(arr):
    """uint32 (n, 16) -> list of oracle points (None for (0, 0))."""
    vals = limbs_to_ints(np.asarray(arr, dtype=np.uint32).reshape(-1, 8))
    return [g1.decode((vals[2 * i], vals[2 * i + 1])) for i in range(len(vals) // 2)]


def points_to_host(pts):
    vals = []
    for pt in pts:
        x, y = g1.encode(pt)
        vals += [x, y]
    return ints_to_limbs(vals).reshape(len(pts), 16)


def fr_from_host(arr):
    return limbs_to_ints(np.asarray(arr, dtype=np.uint32).reshape(-1, 8))
