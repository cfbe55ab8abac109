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


def half_to_full(d, n, Sh):
    """Upper-half couplings [H][NV] -> full stencils [NV][3^d] (diagonal =
    minus the sum of the couplings), by the documented symmetry."""
    nv = n + 1
    NV = nv ** d
    ns = 3 ** d
    c = ns // 2
    S = np.zeros((NV, ns))
    idx = np.arange(NV)
    coords = [(idx // nv ** m) % nv for m in range(d)]
    for j, oi in enumerate(O.half_offsets(d)):
        o = [(oi // 3 ** m) % 3 - 1 for m in range(d)]
        S[:, oi] = Sh[j]
        # the coupling of w = v + o back to v sits at index ns-1-oi of w
        inside = np.ones(NV, bool)
        w = np.zeros(NV, np.int64)
        for m in range(d):
            y = coords[m] + o[m]
            inside &= (y >= 0) & (y <= n)
            w += np.clip(y, 0, n) * nv ** m
        S[w[inside], ns - 1 - oi] = Sh[j][inside]
    S[:, c] = -(S.sum(1) - S[:, c])
    return S
