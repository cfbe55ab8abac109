"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method itself: it only draws the
random material layouts (balls, boxes, Gaussian-field lattices), names the
analytic material laws by parameters, and builds the right-hand-side load
vectors that a caller hands to a solver.  Evaluating a material law at a
point, integrating element matrices and everything after that is done
separately by each side.

Material descriptor (``Field``), one of:

``CONST``   eps = p0
``SINE``    eps = 1 + p0 * prod_m sin(2 pi x_m)
``THETA``   eps = 1 + (0.3/d) prod_m exp(-p0 x_m) cos(pi p0 x_m)
            (the first test setup of the paper's results section, p0 = theta)
``BALLS``   eps = p1 inside any ball |x - c|^2 <= r^2, else p0;
            data = [count][d+1] rows (c_0 .. c_{d-1}, r)
``LATTICE`` eps = exp(p0 * g(x)), g the d-linear interpolant of lattice
            values on a (count+1)^d vertex lattice of spacing 1/count,
            x fastest; data = those values
``BOXES``   eps = value of the last box (in array order) with
            lo_m <= x_m < hi_m for all m, else p0;
            data = [count][2d+1] rows (lo_0.., hi_0.., eps)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

CONST, SINE, THETA, BALLS, LATTICE, BOXES = 0, 1, 2, 3, 4, 5
KIND_NAMES = {CONST: "const", SINE: "sine", THETA: "theta", BALLS: "balls",
              LATTICE: "lattice", BOXES: "boxes"}

# seeds: field seed = 20050360 + config index; serving request i uses 1_000_000 + i
SEED_BASE = 20050360


@dataclass
class Field:
    kind: int
    dim: int
    p0: float = 0.0
    p1: float = 0.0
    count: int = 0
    data: np.ndarray = dc_field(default_factory=lambda: np.zeros(0, np.float64))

    def __post_init__(self):
        self.data = np.ascontiguousarray(self.data, dtype=np.float64).ravel()

    @property
    def name(self):
        return KIND_NAMES[self.kind]


def const_field(dim, value=1.0):
    return Field(CONST, dim, p0=float(value))


def sine_field(dim, amplitude=0.9):
    """eps = 1 + a prod sin(2 pi x_m); a = 0.9 gives eps in [0.1, 1.9] (2D)."""
    return Field(SINE, dim, p0=float(amplitude))


def theta_field(dim, theta):
    return Field(THETA, dim, p0=float(theta))


def balls_field(dim, count, seed, r_lo=0.005, r_hi=0.05, eps_bg=1.0, eps_in=1e3):
    """Union of `count` balls with centres U[0,1]^d and radii U[r_lo, r_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.0, 1.0, size=(count, dim))
    r = rng.uniform(r_lo, r_hi, size=(count, 1))
    return Field(BALLS, dim, p0=float(eps_bg), p1=float(eps_in), count=count,
                 data=np.hstack([c, r]))


def gaussian_lattice(dim, L, seed, corr_len=1.0 / 32.0):
    """White noise on an (L+1)^d vertex lattice, Gaussian-filtered so that the
    covariance is exp(-r^2 / (2 corr_len^2)) (kernel std corr_len/sqrt 2),
    renormalised to zero mean and unit sample standard deviation."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(size=(L + 1,) * dim)
    sig = (corr_len / math.sqrt(2.0)) * L
    g = gaussian_filter(w, sigma=sig, mode="wrap", truncate=4.0)
    g = (g - g.mean()) / g.std()
    # numpy arrays are indexed [z][y][x] so that ravel() is x fastest
    return np.ascontiguousarray(g, dtype=np.float64)


def lattice_field(dim, L, seed, sigma=1.0, corr_len=1.0 / 32.0):
    g = gaussian_lattice(dim, L, seed, corr_len)
    return Field(LATTICE, dim, p0=float(sigma), count=L, data=g.ravel())


def boxes_field(dim, count, seed, side_lo=1.0 / 64, side_hi=1.0 / 8,
                log10_lo=-4.0, log10_hi=4.0, eps_bg=1.0):
    """Random axis-aligned boxes, centres U[0,1]^d, sides U[side_lo, side_hi],
    eps log-uniform in [10^log10_lo, 10^log10_hi]; later boxes paint over
    earlier ones."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.0, 1.0, size=(count, dim))
    half = 0.5 * rng.uniform(side_lo, side_hi, size=(count, dim))
    e = 10.0 ** rng.uniform(log10_lo, log10_hi, size=(count, 1))
    return Field(BOXES, dim, p0=float(eps_bg), count=count,
                 data=np.hstack([c - half, c + half, e]))


# ---------------------------------------------------------------- workloads
def config_field(index, dim=None, n=None):
    """The material law of workload `index` (0-based, in the order listed in
    the design notes): 0 = 2D sine, 1 = 2D balls, 2 = 3D Gaussian field,
    4 = 3D boxes.  Lattice resolution follows the grid (L = n)."""
    seed = SEED_BASE + index
    if index == 0:
        return sine_field(2, 0.9)
    if index == 1:
        return balls_field(dim or 2, 200, seed)
    if index == 2:
        return lattice_field(dim or 3, n or 256, seed, sigma=1.0)
    if index == 4:
        return boxes_field(dim or 3, 512, seed)
    raise ValueError(index)


# ---------------------------------------------------------------- serving
SERVE_SEED_BASE = 1_000_000
SERVE_N = {2: (128, 256, 512, 768, 1024), 3: (64, 96, 128, 160, 192)}


def serving_request(i, sizes=None, lattice=None):
    """Request `i` of the serving workload: dimension 2 or 3 with equal odds,
    grid size uniform over `sizes[dim]`, eps = exp(sigma g) with sigma
    uniform in [0.5, 2] and g a Gaussian field of correlation length 1/32 on
    an L^d lattice (L = `lattice[dim]`, default 128 in 2D and 64 in 3D,
    which resolves the correlation length with 2-4 lattice steps)."""
    sizes = sizes or SERVE_N
    lattice = lattice or {2: 128, 3: 64}
    rng = np.random.Generator(np.random.PCG64(SERVE_SEED_BASE + i))
    dim = 2 if rng.uniform() < 0.5 else 3
    n = int(sizes[dim][rng.integers(len(sizes[dim]))])
    sigma = float(rng.uniform(0.5, 2.0))
    fseed = int(rng.integers(1 << 62))
    return dim, n, lattice_field(dim, lattice[dim], fseed, sigma=sigma)


def poisson_arrivals(count, rate, seed):
    """Arrival times (s) of a Poisson process of `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# ------------------------------------------------------------- load vectors
def n_vertices(dim, n):
    return (n + 1) ** dim


def _grid_coords(dim, n):
    x = np.arange(n + 1, dtype=np.float64) / n
    mesh = np.meshgrid(*([x] * dim), indexing="ij")
    # index order [x, y, z] -> flatten with x fastest
    return [m.transpose(tuple(range(dim))[::-1]).ravel() for m in mesh]


def interior_mask(dim, n):
    idx = np.arange(n + 1)
    inner = (idx > 0) & (idx < n)
    m = inner
    for _ in range(dim - 1):
        m = np.multiply.outer(inner, m)
    return m.ravel().astype(bool)


def load_const(dim, n, fval=1.0):
    """f_h[i] = integral of fval * phi_i = fval * h^d at interior vertices."""
    h = 1.0 / n
    f = np.zeros(n_vertices(dim, n))
    f[interior_mask(dim, n)] = fval * h ** dim
    return f


def load_sine(dim, n):
    """Consistent load of f = d pi^2 prod sin(pi x_m), the right-hand side of
    u = prod sin(pi x_m) for eps = 1; each factor integrates in closed form
    against a hat function: 2 (1 - cos(pi h)) / (pi^2 h) * sin(pi x_i)."""
    h = 1.0 / n
    c = 2.0 * (1.0 - math.cos(math.pi * h)) / (math.pi ** 2 * h)
    xs = _grid_coords(dim, n)
    f = dim * math.pi ** 2 * np.ones(n_vertices(dim, n))
    for x in xs:
        f *= c * np.sin(math.pi * x)
    f[~interior_mask(dim, n)] = 0.0
    return f


def load_quadrature(dim, n, fun, order=3):
    """f_h[i] = integral of fun * phi_i by tensor Gauss-Legendre with `order`
    points per axis per cell (for smooth fun; small grids only).
    fun takes a list of coordinate arrays and returns values."""
    gp, gw = np.polynomial.legendre.leggauss(order)
    gp = 0.5 * (gp + 1.0)
    gw = 0.5 * gw
    h = 1.0 / n
    nv = n + 1
    f = np.zeros(nv ** dim)
    cells = np.stack(np.meshgrid(*([np.arange(n)] * dim), indexing="ij"), -1).reshape(-1, dim)
    for qi in np.ndindex(*([order] * dim)):
        xi = np.array([gp[k] for k in qi])
        w = np.prod([gw[k] for k in qi]) * h ** dim
        pts = [(cells[:, m] + xi[m]) * h for m in range(dim)]
        val = fun(pts) * w
        for a in range(2 ** dim):
            bits = [(a >> m) & 1 for m in range(dim)]
            phi = np.prod([xi[m] if bits[m] else 1.0 - xi[m] for m in range(dim)])
            vid = np.zeros(len(cells), dtype=np.int64)
            stride = 1
            for m in range(dim):
                vid += (cells[:, m] + bits[m]) * stride
                stride *= nv
            np.add.at(f, vid, val * phi)
    f[~interior_mask(dim, n)] = 0.0
    return f


def noise_guess(dim, n, seed, hi=4.0 / 3.0):
    """Initial iterate with interior values U[0, hi] and zero boundary (the
    paper initialises its runs with noise from [0, 4/3])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, hi, size=n_vertices(dim, n))
    u[~interior_mask(dim, n)] = 0.0
    return u
