"""The Python binding checks every caller buffer (dtype, element count,
contiguity, device) before a raw pointer reaches the C ABI, which cannot
check them: a short or mistyped buffer would otherwise be read or written
out of bounds on the device.  These run on the CPU: every check fires before
any library call."""
import numpy as np
import pytest
import torch

import paper_2005_03606_amd as P
import workload as W


class _Ctx:
    """Stands in for a context: the checks only read its device index."""
    device = 0
    h = None


class _Hier(P.Hierarchy):
    """A hierarchy's geometry without a device (levels n, n/2, ...)."""

    def __init__(self, dim, n, precision=P.FP64):
        self.ctx, self.dim, self.n, self.precision = _Ctx(), dim, n, precision
        self.vdtype = torch.float64 if precision == P.FP64 else torch.float32
        self.h = None

    @property
    def nlev(self):
        return 3

    def level_n(self, l):
        return self.n >> l

    def close(self):
        pass


def _raises(fn, *a, **kw):
    with pytest.raises(P.MgdError) as e:
        fn(*a, **kw)
    assert e.value.code == P.EINVAL
    return str(e.value)


def test_field_data_must_match_its_count():
    fld = W.balls_field(2, 5, 1)
    P.Eps(fld, device="cpu")
    bad = W.Field(fld.kind, 2, p0=1.0, p1=2.0, count=6, data=fld.data)
    assert "data values" in _raises(P.Eps, bad, device="cpu")
    lat = W.lattice_field(3, 4, 2)
    P.Eps(lat, device="cpu")
    bad = W.Field(lat.kind, 3, p0=1.0, count=5, data=lat.data)
    _raises(P.Eps, bad, device="cpu")
    box = W.boxes_field(3, 4, 2)
    bad = W.Field(box.kind, 3, p0=1.0, count=4, data=box.data[:-1])
    _raises(P.Eps, bad, device="cpu")


def test_solve_checks_load_and_iterate():
    d, n = 2, 8
    eps = P.Eps(W.sine_field(2), device="cpu")
    nv = (n + 1) ** d
    assert "float64" in _raises(P.solve, _Ctx(), d, n, eps, torch.zeros(nv, dtype=torch.float32))
    assert "elements" in _raises(P.solve, _Ctx(), d, n, eps, torch.zeros(nv - 1, dtype=torch.float64))
    assert "device" in _raises(P.solve, _Ctx(), d, n, eps, torch.zeros(nv, dtype=torch.float64))
    f = torch.zeros(nv, dtype=torch.float64)
    _raises(P.solve, _Ctx(), d, n, eps, f, u=torch.zeros(nv + 1, dtype=torch.float64))
    _raises(P.solve, _Ctx(), 3, n, eps, f)  # eps of another dimension
    strided = torch.zeros(2 * nv, dtype=torch.float64)[::2]
    assert "contiguous" in _raises(P.solve, _Ctx(), d, n, eps, strided)


def test_assemble_checks_cells_samples_and_old_matrices():
    d, n, s = 2, 4, 2
    eps = P.Eps(W.sine_field(2), device="cpu")
    _raises(P.assemble_cells, _Ctx(), d, n, s, eps, cells=torch.zeros(3, dtype=torch.int32))
    _raises(P.assemble_cells, _Ctx(), d, n, s, eps, K_old=torch.zeros(n * n * 6, dtype=torch.float32))
    _raises(P.assemble_cells, _Ctx(), d, n, s, eps, mode=P.MIXED, K_old=torch.zeros(n * n * 6 - 1,
                                                                                        dtype=torch.float32))
    _raises(P.assemble_cells, _Ctx(), 3, n, s, eps)
    _raises(P.assemble_cells, _Ctx(), d, n, s, eps, mode=7)
    with pytest.raises(P.MgdError):
        P.Eps.samples(2, torch.zeros(8, dtype=torch.float32))


def test_gather_checks_element_matrices():
    d, n = 3, 4
    _raises(P.gather_stencils, _Ctx(), d, n, torch.zeros(n ** 3 * 28 - 1, dtype=torch.float64))
    _raises(P.gather_stencils, _Ctx(), d, n, torch.zeros(n ** 3 * 28, dtype=torch.float64), k_mode=P.MIXED)


def test_hierarchy_pieces_check_vectors_per_level():
    h = _Hier(2, 16, P.MIXED)
    f32 = torch.float32
    nv0, nv1 = 17 * 17, 9 * 9
    _raises(h.smooth, 0, torch.zeros(nv0, dtype=torch.float64), torch.zeros(nv0, dtype=f32))
    _raises(h.smooth, 1, torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32))
    _raises(h.smooth, 5, torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32))
    _raises(h.restrict, 0, torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32))
    _raises(h.prolong_add, 0, torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32))
    _raises(h.restrict, 2, torch.zeros(5 * 5, dtype=f32), torch.zeros(3 * 3, dtype=f32))  # no level 3
    _raises(h.presmooth_restrict, 0, None, torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32),
            torch.zeros(nv0, dtype=f32))
    _raises(h.residual, 1, torch.zeros(nv1, dtype=f32), torch.zeros(nv1, dtype=f32), torch.zeros(nv1 + 1, dtype=f32))
    _raises(h.outer_residual, torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32), torch.zeros(nv0, dtype=f32))
    _raises(h.compress, torch.zeros(4 * nv0, dtype=f32), torch.zeros(16 * 16 + 1, dtype=f32))
    _raises(h.compress, torch.zeros(4 * nv0, dtype=torch.float64), torch.zeros(16 * 16, dtype=f32))
    h64 = _Hier(3, 8)
    _raises(h64.set_fine, torch.zeros(13 * 9 ** 3 - 1, dtype=torch.float64))
    _raises(h64.vcycle, torch.zeros(9 ** 3, dtype=torch.float32), torch.zeros(9 ** 3, dtype=torch.float32))


def test_correct_host_buffers_fail_only_for_being_on_the_host():
    """Right dtype and size but host memory: still refused (pointers cross
    the C ABI as device addresses)."""
    h = _Hier(2, 16)
    u = torch.zeros(17 * 17, dtype=torch.float64)
    msg = _raises(h.smooth, 0, u, u.clone())
    assert "device" in msg
