"""CPU FP64 oracle of delayed approximate matrix assembly in multigrid.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the HIP path.  The arithmetic
lives in ``oracle.c`` (plain C, FP64, no blocking or fusion); this module
builds it with gcc, loads it with ctypes and adds numpy conveniences.

Layouts (documented conventions, identical on both sides):
  * cell c = i + N (j + N k), vertex v = i + (N+1)(j + (N+1) k), x fastest;
  * element matrix K_c[a][b], local vertex a with bit m = offset along axis m;
  * full stencils S[v][o], o in {-1,0,1}^d with index sum_m (o_m+1) 3^m.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ENOCONV, EDIVERGED = 0, -4, -5
STATIONARY, PCG = 0, 1


def build(force=False):
    """Compile oracle.c with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC",
                           "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("count", C.c_int32),
                ("pad", C.c_int32), ("p0", C.c_double), ("p1", C.c_double),
                ("data", C.POINTER(C.c_double))]


class Opts(C.Structure):
    _fields_ = [("s_fixed", C.c_int32), ("s_max", C.c_int32), ("lazy", C.c_int32),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("coarsest", C.c_int32),
                ("max_cycles", C.c_int32), ("transfer", C.c_int32),
                ("outer", C.c_int32), ("start", C.c_int32), ("cycle", C.c_int32), ("pad", C.c_int32),
                ("C", C.c_double), ("omega", C.c_double), ("tol", C.c_double),
                ("div_factor", C.c_double)]


class Report(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("status", C.c_int32), ("nlev", C.c_int32),
                ("pad", C.c_int32), ("r0", C.c_double), ("r_final", C.c_double),
                ("cells_at_s", C.c_int64 * 5), ("integrations", C.c_int64),
                ("hist", C.c_double * 512)]


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_F = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        fp = C.POINTER(_Field)
        L.orc_eps.argtypes = [fp, _D]
        L.orc_eps.restype = C.c_double
        L.orc_subcell_matrix.argtypes = [C.c_int, C.c_int, _I32, C.c_double, _D]
        L.orc_element_matrix.argtypes = [fp, C.c_int, C.c_int, C.c_int, C.c_int64, _D]
        L.orc_element_matrix_samples.argtypes = [C.c_int, C.c_int, C.c_int, _D, _D]
        L.orc_assemble.argtypes = [fp, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int64, _D]
        L.orc_ladder_cell.argtypes = [fp, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_double, _D, _D]
        L.orc_ladder_cell.restype = C.c_int
        L.orc_ladder.argtypes = [fp, C.c_int, C.c_int, C.c_int, C.c_double, _D, _I32, _D]
        L.orc_stencils.argtypes = [C.c_int, C.c_int, _D, _D]
        L.orc_base_coupling.argtypes = [C.c_int, C.c_int, _F, C.c_int64, C.c_int,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_half_value.argtypes = [C.c_uint16]
        L.orc_half_value.restype = C.c_double
        L.orc_e4m3_value.argtypes = [C.c_uint8]
        L.orc_e4m3_value.restype = C.c_double
        L.orc_scale_exponent.argtypes = [C.c_double, C.c_int]
        L.orc_scale_exponent.restype = C.c_int
        L.orc_choose_tier.argtypes = [_F, C.c_int, C.c_double, C.c_int, C.c_int]
        L.orc_choose_tier.restype = C.c_int
        L.orc_encode_stencil.argtypes = [_F, C.c_int, C.c_int, _U32]
        L.orc_encode_stencil.restype = C.c_int
        L.orc_decode_entry.argtypes = [C.c_int, C.c_int, C.c_uint32]
        L.orc_decode_entry.restype = C.c_double
        L.orc_galerkin.argtypes = [C.c_int, C.c_int, _D, _D, _D]
        L.orc_transfer_weights.argtypes = [C.c_int, C.c_int, _D, C.c_int, _D]
        L.orc_residual.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D]
        L.orc_jacobi.argtypes = [C.c_int, C.c_int, _D, _D, _D, C.c_double, _D]
        L.orc_restrict.argtypes = [C.c_int, C.c_int, _D, _D, _D]
        L.orc_prolong_add.argtypes = [C.c_int, C.c_int, _D, _D, _D]
        L.orc_dense_matrix.argtypes = [C.c_int, C.c_int, _D, C.c_void_p]
        L.orc_dense_matrix.restype = C.c_int64
        L.orc_cholesky.argtypes = [C.c_int64, _D]
        L.orc_cholesky.restype = C.c_int
        L.orc_cholesky_solve.argtypes = [C.c_int64, _D, _D]
        L.orc_mg_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _D]
        L.orc_mg_level_weights.argtypes = [C.c_void_p, C.c_int]
        L.orc_mg_level_weights.restype = C.POINTER(C.c_double)
        L.orc_mg_create.restype = C.c_void_p
        L.orc_mg_set_fine.argtypes = [C.c_void_p, _D]
        L.orc_mg_set_geometric.argtypes = [C.c_void_p, _D, _D]
        L.orc_mg_levels.argtypes = [C.c_void_p]
        L.orc_mg_level_n.argtypes = [C.c_void_p, C.c_int]
        L.orc_mg_level_stencils.argtypes = [C.c_void_p, C.c_int]
        L.orc_mg_level_stencils.restype = C.POINTER(C.c_double)
        L.orc_mg_destroy.argtypes = [C.c_void_p]
        L.orc_mg_vcycle.argtypes = [C.c_void_p, _D, _D, C.c_double, C.c_int, C.c_int]
        L.orc_mg_adafac.argtypes = [C.c_void_p, _D, _D, C.c_double, C.c_int]
        L.orc_norm_interior.argtypes = [C.c_int, C.c_int, _D]
        L.orc_norm_interior.restype = C.c_double
        L.orc_solve.argtypes = [fp, C.c_int, C.c_int, _D, _D, C.POINTER(Opts), C.POINTER(Report)]
        L.orc_solve.restype = C.c_int
        _lib = L
    return _lib


class _FieldRef:
    """Keeps the numpy data alive while the C struct points at it."""

    def __init__(self, fld):
        self.data = np.ascontiguousarray(fld.data, dtype=np.float64)
        if self.data.size == 0:
            self.data = np.zeros(1)
        self.s = _Field(fld.kind, fld.dim, fld.count, 0, fld.p0, fld.p1,
                        self.data.ctypes.data_as(C.POINTER(C.c_double)))

    @property
    def ptr(self):
        return C.byref(self.s)


def nst(d):
    return 9 if d == 2 else 27


def nvert(d, n):
    return (n + 1) ** d


def ncell(d, n):
    return n ** d


# ------------------------------------------------------------------ wrappers
def eps_at(fld, x):
    r = _FieldRef(fld)
    return lib().orc_eps(r.ptr, np.ascontiguousarray(x, dtype=np.float64))


def subcell_matrix(d, s, q, h):
    G = np.zeros((1 << d) ** 2)
    lib().orc_subcell_matrix(d, s, np.ascontiguousarray(q, dtype=np.int32), h, G)
    return G.reshape(1 << d, 1 << d)


def element_matrix(fld, d, n, s, cell):
    K = np.zeros((1 << d) ** 2)
    r = _FieldRef(fld)
    lib().orc_element_matrix(r.ptr, d, n, s, cell, K)
    return K.reshape(1 << d, 1 << d)


def element_matrix_samples(d, n, s, eps_q):
    K = np.zeros((1 << d) ** 2)
    lib().orc_element_matrix_samples(d, n, s, np.ascontiguousarray(eps_q, dtype=np.float64), K)
    return K.reshape(1 << d, 1 << d)


def assemble(fld, d, n, s, cells=None):
    """Element matrices [len(cells)][2^d][2^d] at sub-sampling s."""
    r = _FieldRef(fld)
    if cells is None:
        cnt = ncell(d, n)
        ptr = None
    else:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        cnt = len(cells)
        ptr = cells.ctypes.data
    K = np.zeros(cnt * (1 << d) ** 2)
    lib().orc_assemble(r.ptr, d, n, s, ptr, cnt, K)
    return K.reshape(cnt, 1 << d, 1 << d)


def ladder(fld, d, n, s_max, C_thr):
    """Adaptive ladder over every cell: (K_final, s_final, rel[cells][4])."""
    r = _FieldRef(fld)
    nc = ncell(d, n)
    K = np.zeros(nc * (1 << d) ** 2)
    sf = np.zeros(nc, np.int32)
    rel = np.full(nc * 4, np.nan)
    lib().orc_ladder(r.ptr, d, n, s_max, C_thr, K, sf, rel)
    return K.reshape(nc, 1 << d, 1 << d), sf, rel.reshape(nc, 4)


def stencils(d, n, K):
    S = np.zeros(nvert(d, n) * nst(d))
    lib().orc_stencils(d, n, np.ascontiguousarray(K, dtype=np.float64).ravel(), S)
    return S.reshape(nvert(d, n), nst(d))


def base_coupling(d, n, eps_c, v, oi):
    b, ref = C.c_double(), C.c_double()
    lib().orc_base_coupling(d, n, np.ascontiguousarray(eps_c, dtype=np.float32), v, oi,
                            C.byref(b), C.byref(ref))
    return b.value, ref.value


GEOMETRIC, BOXMG = 0, 1


def transfer_weights(d, nf, Sf, kind=GEOMETRIC):
    """Prolongation weights [NV_fine][2^d] toward the coarse box corners."""
    Pw = np.zeros(nvert(d, nf) << d)
    lib().orc_transfer_weights(d, nf, np.ascontiguousarray(Sf, dtype=np.float64).ravel(), kind, Pw)
    return Pw.reshape(nvert(d, nf), 1 << d)


def galerkin(d, nf, Sf, Pw=None, kind=GEOMETRIC):
    nc = nf // 2
    if Pw is None:
        Pw = transfer_weights(d, nf, Sf, kind)
    Sc = np.zeros(nvert(d, nc) * nst(d))
    lib().orc_galerkin(d, nf, np.ascontiguousarray(Sf, dtype=np.float64).ravel(),
                       np.ascontiguousarray(Pw, dtype=np.float64).ravel(), Sc)
    return Sc.reshape(nvert(d, nc), nst(d))


def residual(d, n, S, u, f):
    r = np.zeros(nvert(d, n))
    lib().orc_residual(d, n, np.ascontiguousarray(S).ravel(), np.ascontiguousarray(u),
                       np.ascontiguousarray(f), r)
    return r


def jacobi(d, n, S, u, f, omega):
    out = np.zeros(nvert(d, n))
    lib().orc_jacobi(d, n, np.ascontiguousarray(S).ravel(), np.ascontiguousarray(u),
                     np.ascontiguousarray(f), omega, out)
    return out


def _geo_weights(d, nf):
    return transfer_weights(d, nf, np.zeros(nvert(d, nf) * nst(d)), GEOMETRIC)


def restrict(d, nf, r, Pw=None):
    fc = np.zeros(nvert(d, nf // 2))
    Pw = _geo_weights(d, nf) if Pw is None else Pw
    lib().orc_restrict(d, nf, np.ascontiguousarray(Pw, dtype=np.float64).ravel(),
                       np.ascontiguousarray(r), fc)
    return fc


def prolong_add(d, nf, ec, u, Pw=None):
    u = np.array(u, dtype=np.float64, copy=True)
    Pw = _geo_weights(d, nf) if Pw is None else Pw
    lib().orc_prolong_add(d, nf, np.ascontiguousarray(Pw, dtype=np.float64).ravel(),
                          np.ascontiguousarray(ec), u)
    return u


def dense_matrix(d, n, S):
    S = np.ascontiguousarray(S).ravel()
    m = lib().orc_dense_matrix(d, n, S, None)
    A = np.zeros(m * m)
    lib().orc_dense_matrix(d, n, S, A.ctypes.data)
    return A.reshape(m, m)


def cholesky_solve(A, b):
    m = A.shape[0]
    L = np.ascontiguousarray(A, dtype=np.float64).copy().ravel()
    if lib().orc_cholesky(m, L) != 0:
        raise np.linalg.LinAlgError("not positive definite")
    x = np.ascontiguousarray(b, dtype=np.float64).copy()
    lib().orc_cholesky_solve(m, L, x)
    return x


def norm_interior(d, n, r):
    return lib().orc_norm_interior(d, n, np.ascontiguousarray(r, dtype=np.float64))


class Hierarchy:
    """Galerkin hierarchy built from fine full stencils; V-cycles on it."""

    def __init__(self, d, n, S0, coarsest=2, transfer=GEOMETRIC):
        self.d, self.n = d, n
        self.h = lib().orc_mg_create(d, n, coarsest, transfer, np.ascontiguousarray(S0).ravel())

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mg_destroy(self.h)
            self.h = None

    @property
    def nlev(self):
        return lib().orc_mg_levels(self.h)

    def level_n(self, l):
        return lib().orc_mg_level_n(self.h, l)

    def level_stencils(self, l):
        n = self.level_n(l)
        p = lib().orc_mg_level_stencils(self.h, l)
        return np.ctypeslib.as_array(p, shape=(nvert(self.d, n) * nst(self.d),)).copy().reshape(
            nvert(self.d, n), nst(self.d))

    def level_weights(self, l):
        n = self.level_n(l)
        p = lib().orc_mg_level_weights(self.h, l)
        return np.ctypeslib.as_array(p, shape=(nvert(self.d, n) << self.d,)).copy().reshape(
            nvert(self.d, n), 1 << self.d)

    def set_fine(self, S0):
        lib().orc_mg_set_fine(self.h, np.ascontiguousarray(S0).ravel())

    def set_geometric(self, S0, eps_c0):
        """Finest level S0; coarser levels rediscretised from child-averaged
        cell values (finest: eps_c0 per fine cell), d-linear transfers."""
        lib().orc_mg_set_geometric(self.h, np.ascontiguousarray(S0, dtype=np.float64).ravel(),
                                   np.ascontiguousarray(eps_c0, dtype=np.float64).ravel())

    def adafac(self, u, f, omega=0.6, variant=1):
        """One additive adaFAC cycle (variant 1: PI, 2: Jac) from u."""
        u = np.array(u, dtype=np.float64, copy=True)
        lib().orc_mg_adafac(self.h, u, np.ascontiguousarray(f, dtype=np.float64), omega, variant)
        return u

    def vcycle(self, u, f, omega=0.6, nu1=2, nu2=2):
        u = np.array(u, dtype=np.float64, copy=True)
        lib().orc_mg_vcycle(self.h, u, np.ascontiguousarray(f, dtype=np.float64), omega, nu1, nu2)
        return u


def solve(fld, d, n, f, u0=None, s_fixed=0, s_max=16, lazy=False, C_thr=0.01, omega=0.6,
          nu1=2, nu2=2, coarsest=2, tol=1e-10, max_cycles=200, div_factor=100.0,
          transfer=GEOMETRIC, outer=0, start=0, cycle=0):
    """start: after an operator change 0 carries the iterate over (the
    paper), 1 takes the carried iterate or the zero start, whichever has the
    smaller residual on the new operator.  cycle: 0 multiplicative V(nu1,nu2),
    1 additive adaFAC-PI, 2 adaFAC-Jac (stationary outer iteration)."""
    r = _FieldRef(fld)
    u = np.zeros(nvert(d, n)) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    op = Opts(s_fixed, s_max, int(lazy), nu1, nu2, coarsest, max_cycles, transfer, outer, start, cycle, 0,
              C_thr, omega, tol, div_factor)
    rep = Report()
    st = lib().orc_solve(r.ptr, d, n, np.ascontiguousarray(f, dtype=np.float64), u,
                         C.byref(op), C.byref(rep))
    hist = np.array(rep.hist[: min(rep.cycles + 1, 512)])
    return u, dict(status=st, cycles=rep.cycles, r0=rep.r0, r_final=rep.r_final,
                   nlev=rep.nlev, cells_at_s=list(rep.cells_at_s),
                   integrations=rep.integrations, hist=hist)


# ----------------------------------------------------- encoder conveniences
def choose_tier(delta, tau, min_tier, max_tier):
    d = np.ascontiguousarray(delta, dtype=np.float32)
    return lib().orc_choose_tier(d, len(d), tau, min_tier, max_tier)


def encode_stencil(delta, tier):
    d = np.ascontiguousarray(delta, dtype=np.float32)
    words = np.zeros(len(d), np.uint32)
    e8 = lib().orc_encode_stencil(d, len(d), tier, words)
    return e8, words


def decode_entry(tier, e8, word):
    return lib().orc_decode_entry(tier, e8, int(word))


def scale_exponent(maxabs, tier):
    return lib().orc_scale_exponent(maxabs, tier)


# -------------------------------------------------------- half-stencil view
def half_offsets(d):
    """Stencil offset indices above the centre (the stored half)."""
    c = nst(d) // 2
    return list(range(c + 1, nst(d)))


def to_half(d, S):
    """Full stencils [NV][3^d] -> upper-half couplings [H][NV] (slot-major)."""
    return np.ascontiguousarray(np.asarray(S)[:, half_offsets(d)].T)


def compress(d, n, S32_half, eps_c, min_tier, max_tier, tau_abs, tau_rel):
    """Whole-level encoding: (tile_tier, e8 per vertex, words [NV][H])."""
    NV = nvert(d, n)
    H = nst(d) // 2
    L = lib()
    if not hasattr(L, "_cmp_set"):
        _U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        L.orc_compress.argtypes = [C.c_int, C.c_int, _F, _F, C.c_int, C.c_int, C.c_double,
                                   C.c_double, _U8, _U8, _U32]
        L._cmp_set = True
    tt = np.zeros((NV + 63) // 64, np.uint8)
    e8 = np.zeros(NV, np.uint8)
    words = np.zeros(NV * H, np.uint32)
    L.orc_compress(d, n, np.ascontiguousarray(S32_half, dtype=np.float32).ravel(),
                   np.ascontiguousarray(eps_c, dtype=np.float32), min_tier, max_tier,
                   tau_abs, tau_rel, tt, e8, words)
    return tt, e8, words.reshape(NV, H)


def ladder_cells(fld, d, n, cells, s_max, C_thr):
    """Adaptive ladder of the listed cells only: (K_final [k][2^d][2^d], s_final)."""
    r = _FieldRef(fld)
    nl = 1 << d
    Ks, ss = [], []
    for c in cells:
        K = np.zeros(nl * nl)
        rel = np.zeros(4)
        s = lib().orc_ladder_cell(r.ptr, d, n, int(c), s_max, C_thr, K, rel)
        Ks.append(K.reshape(nl, nl))
        ss.append(s)
    return np.array(Ks), np.array(ss)


def _paper_sigs(L):
    if getattr(L, "_paper_set", False):
        return
    U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
    fp = C.POINTER(_Field)
    L.orc_ladder_cell_inc.argtypes = [fp, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_double, _D, _D]
    L.orc_ladder_cell_inc.restype = C.c_int
    L.orc_p3_encode.argtypes = [C.c_double, C.c_int, U8]
    L.orc_p3_decode.argtypes = [U8, C.c_int]
    L.orc_p3_decode.restype = C.c_double
    L.orc_p3_choose.argtypes = [_D, C.c_int, C.c_double]
    L.orc_p3_choose.restype = C.c_int
    L.orc_paper_table.argtypes = [fp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _D]
    L._paper_set = True


def ladder_cell_inc(fld, d, n, cell, n_max, C_thr):
    """The paper's n -> n + 1 ladder of one cell: (K_final, n_final, rel)."""
    L = lib()
    _paper_sigs(L)
    K = np.zeros((1 << d) ** 2)
    rel = np.full(max(n_max - 1, 1), np.nan)
    s = L.orc_ladder_cell_inc(_FieldRef(fld).ptr, d, n, int(cell), n_max, C_thr, K, rel)
    return K.reshape(1 << d, 1 << d), s, rel


def p3_encode(x, p):
    L = lib()
    _paper_sigs(L)
    out = np.zeros(8, np.uint8)
    L.orc_p3_encode(float(x), int(p), out)
    return out[:p].copy()


def p3_decode(b, p):
    L = lib()
    _paper_sigs(L)
    buf = np.zeros(8, np.uint8)
    buf[:p] = b
    return L.orc_p3_decode(buf, int(p))


def p3_choose(surplus, tau):
    L = lib()
    _paper_sigs(L)
    a = np.ascontiguousarray(surplus, dtype=np.float64).ravel()
    return L.orc_p3_choose(a, a.size, tau)


def paper_table(fld, d, n, C_thr, tau, cycles):
    """Per cycle (max n, mean n, compression) of the paper's ladder and format."""
    L = lib()
    _paper_sigs(L)
    out = np.zeros(3 * cycles)
    L.orc_paper_table(_FieldRef(fld).ptr, d, n, C_thr, tau, cycles, out)
    return out.reshape(cycles, 3)


def pairs(d):
    """(a, b) of the packed upper off-diagonal element-matrix entries."""
    nl = 1 << d
    return [(a, b) for a in range(nl) for b in range(a + 1, nl)]


def pack_pairs(d, K):
    """Full element matrices [k][2^d][2^d] -> packed upper pairs [k][U]."""
    K = np.asarray(K)
    return np.ascontiguousarray(np.stack([K[:, a, b] for a, b in pairs(d)], axis=1))
