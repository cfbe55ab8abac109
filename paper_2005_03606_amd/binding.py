"""ctypes binding of libmgdelay.so (same names as the C ABI, minus the prefix)."""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libmgdelay.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, EDIVERGED, ESTARVED = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
GEOMETRIC, BOXMG = 0, 1
STATIONARY, PCG = 0, 1
UPFRONT, LAZY = 0, 1
PUBLISH_ASYNC, PUBLISH_DETERMINISTIC, PUBLISH_EVERY = 0, 1, 2
STORE_AUTO, STORE_DECODE, STORE_COPY = 0, 1, 2
START_CARRY, START_BEST = 0, 1
CYCLE_V, CYCLE_ADAFAC_PI, CYCLE_ADAFAC_JAC = 0, 1, 2
EPS_SAMPLES = 6
HIST = 512


class MgdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mgd error {code}: {msg}")
        self.code = code


class _Eps(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("count", C.c_int32), ("pad", C.c_int32),
                ("p0", C.c_double), ("p1", C.c_double), ("data", C.c_void_p)]


class _HierDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32), ("precision", C.c_int32),
                ("transfer", C.c_int32), ("coarsest", C.c_int32), ("store_path", C.c_int32)]


class _Tier(C.Structure):
    _fields_ = [("min_tier", C.c_int32), ("max_tier", C.c_int32),
                ("tau_abs", C.c_double), ("tau_rel", C.c_double)]


class _CycleOpts(C.Structure):
    _fields_ = [("omega", C.c_double), ("nu1", C.c_int32), ("nu2", C.c_int32)]


class _SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("transfer", C.c_int32), ("outer", C.c_int32),
                ("schedule", C.c_int32), ("publish", C.c_int32), ("s_fixed", C.c_int32),
                ("s_max", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("max_cycles", C.c_int32), ("coarsest", C.c_int32), ("store_path", C.c_int32),
                ("C", C.c_double), ("omega", C.c_double), ("tol", C.c_double),
                ("div_factor", C.c_double), ("tiers", _Tier), ("prov_tol", C.c_double),
                ("start", C.c_int32), ("cycle", C.c_int32), ("prov_growth", C.c_double)]


class _Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("nlev", C.c_int32),
                ("publishes", C.c_int32), ("checks", C.c_int32), ("pad", C.c_int32),
                ("r0", C.c_double), ("r_final", C.c_double),
                ("cells_at_s", C.c_int64 * 5), ("integrations", C.c_int64),
                ("tier_tiles", C.c_int64 * 4), ("store_bytes", C.c_double),
                ("t_total_ms", C.c_double), ("t_first_cycle_ms", C.c_double),
                ("t_cycles_ms", C.c_double), ("hist", C.c_double * HIST)]


class _ServerOpts(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("pad", C.c_int32), ("hbm_budget_bytes", C.c_double)]


_lib = None
_P = C.c_void_p
_I = C.c_int32


def lib():
    """Load libmgdelay.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(f"{library_path} is missing: build it with paper_2005_03606_amd/build.py "
                           "(there is no CPU fallback)")
    L = C.CDLL(library_path)
    sig = {
        "mgd_create": ([C.POINTER(_P), C.c_int], C.c_int),
        "mgd_destroy": ([_P], C.c_int),
        "mgd_last_error": ([_P], C.c_char_p),
        "mgd_version": ([], C.c_char_p),
        "mgd_assemble_cells": ([_P, _I, _I, _I, _P, C.c_int64, C.POINTER(_Eps), _I, _P, _P,
                                C.c_double, _P, _P, _P], C.c_int),
        "mgd_ladder_step_keep": ([_P, _I, _I, _I, _P, C.c_int64, C.POINTER(_Eps), _P, C.c_double, _P, _P, _P],
                                 C.c_int),
        "mgd_p3_encode": ([_P, _I, _P, _P, C.c_int64, C.c_double, _P, _P, _P], C.c_int),
        "mgd_gather_stencils": ([_P, _I, _I, _P, _I, _P, _I, _P], C.c_int),
        "mgd_centre_samples": ([_P, _I, _I, C.POINTER(_Eps), _P, _P], C.c_int),
        "mgd_hier_create": ([_P, C.POINTER(_HierDesc), C.POINTER(_P)], C.c_int),
        "mgd_hier_destroy": ([_P], C.c_int),
        "mgd_hier_levels": ([_P], C.c_int),
        "mgd_hier_level_n": ([_P, C.c_int], C.c_int),
        "mgd_hier_set_fine": ([_P, _P, _P, _P], C.c_int),
        "mgd_compress_stencils": ([_P, _P, _P, _P, C.POINTER(_Tier), _P], C.c_int),
        "mgd_compress_stencils_noalloc": ([_P, _P, _P, _P, C.POINTER(_Tier), _P], C.c_int),
        "mgd_store_info": ([_P, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64 * 4)], C.c_int),
        "mgd_store_export": ([_P, _P, _P, _P, _P, _P], C.c_int),
        "mgd_weight_tiles": ([_P, _P, _I, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
        "mgd_tier0_items": ([_P, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _P], C.c_int),
        "mgd_coarsen": ([_P, _P, _P], C.c_int),
        "mgd_level_stencils": ([_P, _P, C.c_int, _P, _P], C.c_int),
        "mgd_level_weights": ([_P, _P, C.c_int, _P, _P], C.c_int),
        "mgd_smooth": ([_P, _P, C.c_int, _P, _P, _I, C.c_double, _P], C.c_int),
        "mgd_presmooth": ([_P, _P, _I, _P, _P, _P, _P, C.c_double, _P], C.c_int),
        "mgd_presmooth_restrict": ([_P, _P, _I, _P, _P, _P, _P, C.c_double, _P], C.c_int),
        "mgd_residual": ([_P, _P, C.c_int, _P, _P, _P, _P], C.c_int),
        "mgd_restrict": ([_P, _P, C.c_int, _P, _P, _P], C.c_int),
        "mgd_prolong_add": ([_P, _P, C.c_int, _P, _P, _P], C.c_int),
        "mgd_vcycle": ([_P, _P, _P, _P, C.POINTER(_CycleOpts), _P], C.c_int),
        "mgd_outer_residual": ([_P, _P, _P, _P, _P, _P], C.c_int),
        "mgd_solve": ([_P, _I, _I, C.POINTER(_Eps), _P, _P, C.POINTER(_SolveOpts),
                       C.POINTER(_Report), _P], C.c_int),
        "mgd_solve_footprint": ([_I, _I, C.POINTER(_SolveOpts), C.POINTER(C.c_double)], C.c_int),
        "mgd_server_create": ([_P, C.POINTER(_ServerOpts), C.POINTER(_P)], C.c_int),
        "mgd_server_destroy": ([_P], C.c_int),
        "mgd_server_submit": ([_P, _I, _I, C.POINTER(_Eps), _P, _P, C.POINTER(_SolveOpts), _P,
                               C.POINTER(C.c_int64)], C.c_int),
        "mgd_server_poll": ([_P, C.POINTER(_I), C.POINTER(_I)], C.c_int),
        "mgd_server_result": ([_P, C.c_int64, C.POINTER(_Report), C.POINTER(C.c_double * 3)], C.c_int),
        "mgd_server_stats": ([_P, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(_I)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def n_half(dim):
    return 4 if dim == 2 else 13


def n_pairs(dim):
    return 6 if dim == 2 else 28


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise MgdError(EINVAL, "device tensor expected")
    if not t.is_contiguous():
        raise MgdError(EINVAL, "contiguous tensor expected")
    return t.data_ptr()


_DT = {FP64: torch.float64, MIXED: torch.float32}


def _buf(t, name, dtype, numel, device=None, optional=False):
    """Device pointer of a caller buffer after checking what the C ABI cannot:
    dtype, element count, contiguity, and that it lives on the context's
    device.  Raises MgdError(EINVAL) before anything is enqueued."""
    if t is None:
        if optional:
            return None
        raise MgdError(EINVAL, f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise MgdError(EINVAL, f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise MgdError(EINVAL, f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise MgdError(EINVAL, f"{name} must hold {numel} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise MgdError(EINVAL, f"{name} must be contiguous")
    if not t.is_cuda:
        raise MgdError(EINVAL, f"{name} must be a device tensor")
    if device is not None and t.device.index != device:
        raise MgdError(EINVAL, f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    return t.data_ptr()


def _nv(dim, n):
    return (n + 1) ** dim


def _eps_data_count(kind, dim, count):
    """Doubles a field descriptor's data must hold (None: no data)."""
    if kind == 3:                      # balls: (c, r) rows
        return count * (dim + 1)
    if kind == 4:                      # lattice: (count+1)^d vertex values
        return (count + 1) ** dim
    if kind == 5:                      # boxes: (lo, hi, eps) rows
        return count * (2 * dim + 1)
    return None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """Per-device library context (mgd_create / mgd_destroy)."""

    def __init__(self, device=0):
        L = lib()
        h = _P()
        rc = L.mgd_create(C.byref(h), device)
        if rc != OK:
            raise MgdError(rc, f"mgd_create(device={device}) failed")
        self.h = h
        self.device = device

    def check(self, rc):
        if rc != OK and rc not in (ENOCONV, EDIVERGED, ESTARVED):
            raise MgdError(rc, lib().mgd_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().mgd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Eps:
    """Material descriptor on the device (any object with kind, dim, p0, p1,
    count and a float64 `data` array, e.g. workload.Field)."""

    def __init__(self, field, device="cuda"):
        import numpy as np
        data = np.ascontiguousarray(getattr(field, "data", np.zeros(0)), dtype=np.float64)
        if field.dim not in (2, 3):
            raise MgdError(EINVAL, f"field dim must be 2 or 3, got {field.dim}")
        want = _eps_data_count(field.kind, field.dim, field.count)
        if want is not None and (field.count < 1 or data.size != want):
            raise MgdError(EINVAL, f"field kind {field.kind} with count {field.count} needs {want} data values, "
                                   f"got {data.size}")
        self.data = torch.from_numpy(data if data.size else np.zeros(1)).to(device)
        self.s = _Eps(field.kind, field.dim, field.count, 0, field.p0, field.p1, self.data.data_ptr())
        self.dim = field.dim
        self.n_samples = None

    @classmethod
    def samples(cls, dim, samples):
        """Explicit samples [cells][s^d] (float64, device) for assemble_cells."""
        if samples.dtype != torch.float64:
            raise MgdError(EINVAL, f"samples must be torch.float64, got {samples.dtype}")
        obj = cls.__new__(cls)
        obj.data = samples.contiguous()
        obj.s = _Eps(EPS_SAMPLES, dim, 0, 0, 0.0, 0.0, _ptr(obj.data))
        obj.dim = dim
        obj.n_samples = obj.data.numel()
        return obj


def assemble_cells(ctx, dim, n, s, eps, mode=FP64, cells=None, K_old=None, C_thr=0.01,
                   want_rel=False, stream=None):
    """Element matrices [count][U] (upper off-diagonal pairs); with K_old also
    the relative change and the below-threshold flags."""
    if dim not in (2, 3) or mode not in _DT:
        raise MgdError(EINVAL, "dim must be 2 or 3 and mode FP64 or MIXED")
    if eps.dim != dim:
        raise MgdError(EINVAL, "eps dimension differs from dim")
    ncell = n ** dim
    if cells is None:
        count = ncell
    else:
        count = int(cells.numel())
        _buf(cells, "cells", torch.int64, count, ctx.device)
        if count and (int(cells.min()) < 0 or int(cells.max()) >= ncell):
            raise MgdError(EINVAL, f"cell ids must lie in [0, {ncell})")
    if eps.n_samples is not None and eps.n_samples != count * s ** dim:
        raise MgdError(EINVAL, f"explicit samples must number count * s^d = {count * s ** dim}")
    dev = torch.device("cuda", ctx.device)
    dt = _DT[mode]
    _buf(K_old, "K_old", dt, count * n_pairs(dim), ctx.device, optional=True)
    K = torch.empty((count, n_pairs(dim)), dtype=dt, device=dev)
    rel = torch.empty(count, dtype=torch.float64, device=dev) if (K_old is not None and want_rel) else None
    done = torch.empty(count, dtype=torch.uint8, device=dev) if K_old is not None else None
    ctx.check(lib().mgd_assemble_cells(ctx.h, dim, n, s, _ptr(cells), count, C.byref(eps.s), mode,
                                       _ptr(K), _ptr(K_old), C_thr, _ptr(rel), _ptr(done), _stream(stream)))
    return K, rel, done


def ladder_step_keep(ctx, dim, n, s, eps, K, cells=None, C_thr=0.01, want_rel=False, stream=None):
    """The paper's n -> n + 1 step at s samples per axis (FP64): K (device
    float64 [n^d][U], rows by cell, holding the (s-1)^d-sample matrices of
    the listed cells) keeps a cell's row when it changed by less than C_thr,
    else takes the new matrix.  Returns (rel, done) over the listed cells."""
    if dim not in (2, 3):
        raise MgdError(EINVAL, "dim must be 2 or 3")
    if eps.dim != dim or eps.n_samples is not None:
        raise MgdError(EINVAL, "the ladder step needs a field descriptor of dimension dim")
    ncell = n ** dim
    if cells is None:
        count = ncell
    else:
        count = int(cells.numel())
        _buf(cells, "cells", torch.int64, count, ctx.device)
        if count and (int(cells.min()) < 0 or int(cells.max()) >= ncell):
            raise MgdError(EINVAL, f"cell ids must lie in [0, {ncell})")
    _buf(K, "K", torch.float64, ncell * n_pairs(dim), ctx.device)
    dev = torch.device("cuda", ctx.device)
    rel = torch.empty(count, dtype=torch.float64, device=dev) if want_rel else None
    done = torch.empty(count, dtype=torch.uint8, device=dev)
    ctx.check(lib().mgd_ladder_step_keep(ctx.h, dim, n, s, _ptr(cells), count, C.byref(eps.s), _ptr(K), C_thr,
                                         _ptr(rel), _ptr(done), _stream(stream)))
    return rel, done


def p3_encode(ctx, dim, K, K1, tau, stream=None):
    """The paper's p3-byte format of the surplus K - K1 (device float64
    [count][U] each), cell by cell: (p3 [count] uint8, bytes [count][2^d 2^d 8]
    uint8, of which a cell's first 2^d 2^d p3 bytes are its entries)."""
    if dim not in (2, 3):
        raise MgdError(EINVAL, "dim must be 2 or 3")
    U = n_pairs(dim)
    count = int(K.numel()) // U if K is not None else 0
    _buf(K, "K", torch.float64, count * U, ctx.device)
    _buf(K1, "K1", torch.float64, count * U, ctx.device)
    dev = torch.device("cuda", ctx.device)
    nn = (1 << dim) ** 2
    p3 = torch.empty(count, dtype=torch.uint8, device=dev)
    out = torch.zeros((count, nn * 8), dtype=torch.uint8, device=dev)
    ctx.check(lib().mgd_p3_encode(ctx.h, dim, _ptr(K), _ptr(K1), count, float(tau), _ptr(p3), _ptr(out),
                                  _stream(stream)))
    return p3, out


def centre_samples(ctx, dim, n, eps, stream=None):
    """FP32 eps at every cell centre [n^d]."""
    if eps.dim != dim or eps.n_samples is not None:
        raise MgdError(EINVAL, "centre samples need a field descriptor of dimension dim")
    out = torch.empty(n ** dim, dtype=torch.float32, device=torch.device("cuda", ctx.device))
    ctx.check(lib().mgd_centre_samples(ctx.h, dim, n, C.byref(eps.s), _ptr(out), _stream(stream)))
    return out


def gather_stencils(ctx, dim, n, K, k_mode=FP64, s_mode=FP64, stream=None):
    """Upper-half couplings [H][NV] from element matrices of all cells."""
    if dim not in (2, 3) or k_mode not in _DT or s_mode not in _DT:
        raise MgdError(EINVAL, "dim must be 2 or 3 and the modes FP64 or MIXED")
    _buf(K, "K", _DT[k_mode], n ** dim * n_pairs(dim), ctx.device)
    S = torch.empty((n_half(dim), (n + 1) ** dim), dtype=_DT[s_mode], device=K.device)
    ctx.check(lib().mgd_gather_stencils(ctx.h, dim, n, _ptr(K), k_mode, _ptr(S), s_mode, _stream(stream)))
    return S


class Hierarchy:
    def __init__(self, ctx, dim, n, precision=FP64, transfer=GEOMETRIC, coarsest=2, store_path=STORE_AUTO):
        self.ctx, self.dim, self.n, self.precision = ctx, dim, n, precision
        d = _HierDesc(dim, n, precision, transfer, coarsest, store_path)
        h = _P()
        ctx.check(lib().mgd_hier_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h
        self.vdtype = torch.float64 if precision == FP64 else torch.float32

    def close(self):
        if getattr(self, "h", None):
            lib().mgd_hier_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nlev(self):
        return lib().mgd_hier_levels(self.h)

    def level_n(self, l):
        return lib().mgd_hier_level_n(self.h, l)

    def nv(self, l=0):
        return (self.level_n(l) + 1) ** self.dim

    def vec(self, l=0):
        return torch.zeros(self.nv(l), dtype=self.vdtype, device=torch.device("cuda", self.ctx.device))

    def _level(self, l):
        if not (0 <= l < self.nlev):
            raise MgdError(EINVAL, f"level {l} outside [0, {self.nlev})")
        return l

    def _vec(self, t, name, l, optional=False):
        return _buf(t, name, self.vdtype, self.nv(l), self.ctx.device, optional)

    def set_fine(self, S64, stream=None):
        _buf(S64, "S", torch.float64, n_half(self.dim) * self.nv(0), self.ctx.device)
        self.ctx.check(lib().mgd_hier_set_fine(self.ctx.h, self.h, _ptr(S64), _stream(stream)))

    def compress(self, S32, eps_c, min_tier=2, max_tier=2, tau_abs=0.0, tau_rel=0.0, stream=None):
        _buf(S32, "S32", torch.float32, n_half(self.dim) * self.nv(0), self.ctx.device)
        _buf(eps_c, "eps_c", torch.float32, self.n ** self.dim, self.ctx.device)
        pol = _Tier(min_tier, max_tier, tau_abs, tau_rel)
        self.ctx.check(lib().mgd_compress_stencils(self.ctx.h, self.h, _ptr(S32), _ptr(eps_c),
                                                   C.byref(pol), _stream(stream)))

    def compress_noalloc(self, S32, eps_c, min_tier=2, max_tier=2, tau_abs=0.0, tau_rel=0.0, stream=None):
        """compress() without device allocation (static scratch; bounded level size)."""
        _buf(S32, "S32", torch.float32, n_half(self.dim) * self.nv(0), self.ctx.device)
        _buf(eps_c, "eps_c", torch.float32, self.n ** self.dim, self.ctx.device)
        pol = _Tier(min_tier, max_tier, tau_abs, tau_rel)
        self.ctx.check(lib().mgd_compress_stencils_noalloc(self.ctx.h, self.h, _ptr(S32), _ptr(eps_c),
                                                           C.byref(pol), _stream(stream)))

    def coarsen(self, stream=None):
        self.ctx.check(lib().mgd_coarsen(self.ctx.h, self.h, _stream(stream)))

    def store_info(self):
        nt, pb, tiers = C.c_int64(), C.c_int64(), (C.c_int64 * 4)()
        self.ctx.check(lib().mgd_store_info(self.ctx.h, self.h, C.byref(nt), C.byref(pb), C.byref(tiers)))
        return nt.value, pb.value, list(tiers)

    def weight_tiles(self, level):
        """(tiles, tiles whose BoxMG prolongation is d-linear) of a 3D BoxMG level."""
        nt, geo = C.c_int64(), C.c_int64()
        self.ctx.check(lib().mgd_weight_tiles(self.ctx.h, self.h, level, C.byref(nt), C.byref(geo)))
        return nt.value, geo.value

    def tier0_items(self, stream=None):
        """(items, items re-evaluated from the centre samples) of the default
        3D sweep on the finest level."""
        it, t0 = C.c_int64(), C.c_int64()
        self.ctx.check(lib().mgd_tier0_items(self.ctx.h, self.h, C.byref(it), C.byref(t0), _stream(stream)))
        return it.value, t0.value

    def store_export(self, stream=None):
        nt, pb, _ = self.store_info()
        dev = torch.device("cuda", self.ctx.device)
        tt = torch.empty(nt, dtype=torch.uint8, device=dev)
        off = torch.empty(nt, dtype=torch.int32, device=dev)
        pay = torch.empty(max(pb, 1), dtype=torch.uint8, device=dev)
        self.ctx.check(lib().mgd_store_export(self.ctx.h, self.h, _ptr(tt), _ptr(off), _ptr(pay),
                                              _stream(stream)))
        return tt, off, pay[:pb]

    def level_stencils(self, l, stream=None):
        self._level(l)
        out = torch.empty((n_half(self.dim), self.nv(l)), dtype=torch.float64,
                          device=torch.device("cuda", self.ctx.device))
        self.ctx.check(lib().mgd_level_stencils(self.ctx.h, self.h, l, _ptr(out), _stream(stream)))
        return out

    def level_weights(self, l, stream=None):
        self._level(l)
        out = torch.empty((1 << self.dim, self.nv(l)), dtype=torch.float64,
                          device=torch.device("cuda", self.ctx.device))
        self.ctx.check(lib().mgd_level_weights(self.ctx.h, self.h, l, _ptr(out), _stream(stream)))
        return out

    def smooth(self, l, u, f, sweeps=1, omega=0.6, stream=None):
        self._level(l)
        self._vec(u, "u", l)
        self._vec(f, "f", l)
        self.ctx.check(lib().mgd_smooth(self.ctx.h, self.h, l, _ptr(u), _ptr(f), sweeps, omega, _stream(stream)))

    def presmooth(self, l, u, f, u_out, r_out, omega=0.6, stream=None):
        """Two sweeps from u (None: zero) into u_out, then r_out = f - A u_out."""
        self._level(l)
        self._vec(u, "u", l, optional=True)
        for t, nm in ((f, "f"), (u_out, "u_out"), (r_out, "r_out")):
            self._vec(t, nm, l)
        self.ctx.check(lib().mgd_presmooth(self.ctx.h, self.h, l, _ptr(u), _ptr(f), _ptr(u_out), _ptr(r_out),
                                           omega, _stream(stream)))

    def presmooth_restrict(self, l, u, f, u_out, fc, omega=0.6, stream=None):
        """Two sweeps from u (None: zero) into u_out, fc = P^T (f - A u_out) on level l+1."""
        self._level(l)
        self._level(l + 1)
        self._vec(u, "u", l, optional=True)
        self._vec(f, "f", l)
        self._vec(u_out, "u_out", l)
        self._vec(fc, "fc", l + 1)
        self.ctx.check(lib().mgd_presmooth_restrict(self.ctx.h, self.h, l, _ptr(u), _ptr(f), _ptr(u_out), _ptr(fc),
                                                    omega, _stream(stream)))

    def residual(self, l, u, f, r, stream=None):
        self._level(l)
        for t, nm in ((u, "u"), (f, "f"), (r, "r")):
            self._vec(t, nm, l)
        self.ctx.check(lib().mgd_residual(self.ctx.h, self.h, l, _ptr(u), _ptr(f), _ptr(r), _stream(stream)))

    def restrict(self, l, r, fc, stream=None):
        self._level(l)
        self._level(l + 1)
        self._vec(r, "r", l)
        self._vec(fc, "fc", l + 1)
        self.ctx.check(lib().mgd_restrict(self.ctx.h, self.h, l, _ptr(r), _ptr(fc), _stream(stream)))

    def prolong_add(self, l, ec, u, stream=None):
        self._level(l)
        self._level(l + 1)
        self._vec(ec, "ec", l + 1)
        self._vec(u, "u", l)
        self.ctx.check(lib().mgd_prolong_add(self.ctx.h, self.h, l, _ptr(ec), _ptr(u), _stream(stream)))

    def vcycle(self, u, f, omega=0.6, nu1=2, nu2=2, stream=None):
        self._vec(u, "u", 0)
        self._vec(f, "f", 0)
        o = _CycleOpts(omega, nu1, nu2)
        self.ctx.check(lib().mgd_vcycle(self.ctx.h, self.h, _ptr(u), _ptr(f), C.byref(o), _stream(stream)))

    def outer_residual(self, u, f, r, stream=None):
        for t, nm in ((u, "u"), (f, "f"), (r, "r")):
            _buf(t, nm, torch.float64, self.nv(0), self.ctx.device)
        self.ctx.check(lib().mgd_outer_residual(self.ctx.h, self.h, _ptr(u), _ptr(f), _ptr(r), _stream(stream)))


def solve_opts(precision=FP64, transfer=GEOMETRIC, outer=STATIONARY, schedule=UPFRONT,
               publish=PUBLISH_ASYNC, s_fixed=0, s_max=16, C_thr=0.01, omega=0.6, nu1=2, nu2=2,
               tol=1e-8, max_cycles=200, coarsest=2, div_factor=100.0, min_tier=2, max_tier=2,
               tau_abs=0.0, tau_rel=0.0, prov_tol=0.0, store_path=0, start=START_CARRY, cycle=CYCLE_V,
               prov_growth=0.0):
    return _SolveOpts(precision, transfer, outer, schedule, publish, s_fixed, s_max, nu1, nu2,
                      max_cycles, coarsest, store_path, C_thr, omega, tol, div_factor,
                      _Tier(min_tier, max_tier, tau_abs, tau_rel), prov_tol, start, cycle, prov_growth)


def _report_dict(rc, rep):
    k = rep.checks
    return dict(status=rc, cycles=rep.cycles, nlev=rep.nlev, publishes=rep.publishes, r0=rep.r0,
                r_final=rep.r_final, cells_at_s=list(rep.cells_at_s), integrations=rep.integrations,
                tier_tiles=list(rep.tier_tiles), store_bytes=rep.store_bytes,
                t_total_ms=rep.t_total_ms, t_first_cycle_ms=rep.t_first_cycle_ms,
                t_cycles_ms=rep.t_cycles_ms, hist=list(rep.hist[:k]))


def solve(ctx, dim, n, eps, f, u=None, stream=None, **kw):
    """Full solve (synchronous).  f, u: device float64 [(n+1)^d]; u is the
    initial guess (zero if None) and holds the solution on return.  Keyword
    options as in solve_opts."""
    if eps.dim != dim or eps.n_samples is not None:
        raise MgdError(EINVAL, "solve needs a field descriptor of dimension dim")
    _buf(f, "f", torch.float64, _nv(dim, n), ctx.device)
    if u is None:
        u = torch.zeros_like(f)
    _buf(u, "u", torch.float64, _nv(dim, n), ctx.device)
    op = solve_opts(**kw)
    rep = _Report()
    rc = ctx.check(lib().mgd_solve(ctx.h, dim, n, C.byref(eps.s), _ptr(f), _ptr(u), C.byref(op),
                                   C.byref(rep), _stream(stream)))
    return u, _report_dict(rc, rep)


def solve_footprint(dim, n, **kw):
    b = C.c_double()
    rc = lib().mgd_solve_footprint(dim, n, C.byref(solve_opts(**kw)), C.byref(b))
    if rc != OK:
        raise MgdError(rc, "bad footprint arguments")
    return b.value


class Server:
    """Continuous-batching solve server (mgd_server_*)."""

    def __init__(self, ctx, max_slots=8, budget_bytes=64e9):
        self.ctx = ctx
        h = _P()
        ctx.check(lib().mgd_server_create(ctx.h, C.byref(_ServerOpts(max_slots, 0, budget_bytes)), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, dim, n, eps, f, u, stream=None, **kw):
        """Queue a solve; it starts after the work queued so far on `stream`
        (default: the current torch stream), where f and u were written."""
        if eps.dim != dim or eps.n_samples is not None:
            raise MgdError(EINVAL, "a request needs a field descriptor of dimension dim")
        _buf(f, "f", torch.float64, _nv(dim, n), self.ctx.device)
        _buf(u, "u", torch.float64, _nv(dim, n), self.ctx.device)
        t = C.c_int64()
        op = solve_opts(**kw)
        self.ctx.check(lib().mgd_server_submit(self.h, dim, n, C.byref(eps.s), _ptr(f), _ptr(u),
                                               C.byref(op), _stream(stream), C.byref(t)))
        self._keep[t.value] = (eps, f, u)
        return t.value

    def poll(self):
        a, w = _I(), _I()
        rc = lib().mgd_server_poll(self.h, C.byref(a), C.byref(w))
        if rc < 0:
            raise MgdError(rc, lib().mgd_last_error(self.ctx.h).decode())
        return rc, a.value, w.value

    def result(self, ticket):
        rep = _Report()
        times = (C.c_double * 3)()
        rc = lib().mgd_server_result(self.h, ticket, C.byref(rep), C.byref(times))
        if rc < 0:
            raise MgdError(rc, lib().mgd_last_error(self.ctx.h).decode())
        if rc == 0:
            return None
        keep = self._keep.pop(ticket, None)
        return rep.status, _report_dict(rep.status, rep), tuple(times), keep

    def stats(self):
        c, b, i = C.c_int64(), C.c_double(), _I()
        lib().mgd_server_stats(self.h, C.byref(c), C.byref(b), C.byref(i))
        return dict(completed=c.value, resident_bytes=b.value, idle_states=i.value)

    def close(self):
        if getattr(self, "h", None):
            lib().mgd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
