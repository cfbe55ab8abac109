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


def ulp_perturb(a, rng):
    """a with every nonzero entry moved by one ulp, random sign."""
    a = np.asarray(a, dtype=np.float64)
    return a + rng.choice([-1.0, 1.0], size=a.shape) * np.spacing(np.abs(a)) * (a != 0)


def oracle_spread(run, f, trials=2, seed=0):
    """How far the oracle's own residual history and solution move when the
    load vector changes by one ulp per entry: the size of the differences any
    other correct FP64 implementation (another summation order) produces.
    run(f) -> (u, rep).  Returns ((u, rep) of the unperturbed run,
    hist_floor, u_spread): the largest history change over the checks whose
    value is at most 1e-6 (the rounding floor of the late checks) and the
    largest solution change relative to max |u|."""
    rng = np.random.default_rng(seed)
    u0, r0 = run(f)
    h0 = np.asarray(r0["hist"])
    floor = 0.0
    us = 0.0
    for _ in range(trials):
        u1, r1 = run(ulp_perturb(f, rng))
        h1 = np.asarray(r1["hist"])
        m = min(len(h0), len(h1))
        late = h0[:m] <= 1e-6
        if late.any():
            floor = max(floor, float(np.abs(h0[:m] - h1[:m])[late].max()))
        us = max(us, rel_err(u1, u0))
    return (u0, r0), max(floor, 1e-300), max(us, 1e-300)


def assert_hist_close(got, want, floor, rtol=1e-7, factor=100.0, label=""):
    """Residual histories agree to rtol relative, and down at the rounding
    floor to `factor` times the oracle's own one-ulp spread."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    dev = np.abs(got - want)
    tol = rtol * np.abs(want) + factor * floor
    ratio = float((dev / (rtol * np.abs(want) + floor)).max())
    print(f"{label} hist: max dev {dev.max():.3e}, floor {floor:.3e}, dev/(rtol h + floor) {ratio:.2f}")
    assert (dev <= tol).all(), (dev.max(), floor)
