"""Helpers shared by the GPU tests (not collected)."""
import numpy as np

import oracle as O


def half_mask(d, n):
    """[H][NV] mask of stored couplings with at least one interior endpoint."""
    nv = n + 1
    NV = nv ** d
    offs = []
    for oi in O.half_offsets(d):
        offs.append([(oi // 3 ** m) % 3 - 1 for m in range(d)])
    idx = np.arange(NV)
    coords = [(idx // nv ** m) % nv for m in range(d)]
    inner_v = np.ones(NV, bool)
    for x in coords:
        inner_v &= (x > 0) & (x < n)
    M = np.zeros((len(offs), NV), bool)
    for j, o in enumerate(offs):
        inside = np.ones(NV, bool)
        inner_w = np.ones(NV, bool)
        for m in range(d):
            y = coords[m] + o[m]
            inside &= (y >= 0) & (y <= n)
            inner_w &= (y > 0) & (y < n)
        M[j] = inside & (inner_v | inner_w)
    return M


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)
