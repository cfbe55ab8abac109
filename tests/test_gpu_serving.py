"""Serving loop: each request's result is the same alone and in the mix,
admission respects the device-memory budget, and resident state is reused."""
import numpy as np
import pytest
import torch

import workload as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2005_03606_amd")
from paper_2005_03606_amd import serving  # noqa: E402

SHAPES = [(2, 32), (3, 8), (2, 64), (3, 16), (2, 48), (3, 12)]
BASE = dict(precision=P.MIXED, schedule=P.LAZY, transfer=P.BOXMG, outer=P.PCG, s_max=16, tol=1e-8,
            max_cycles=300, min_tier=2, max_tier=2, tau_rel=1e-7)


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    c.close()


def make_requests(shapes, seed0=0):
    reqs = []
    for k, (d, n) in enumerate(shapes):
        fld = W.lattice_field(d, 32 if d == 2 else 16, 77 + seed0 + k, sigma=0.5 + 0.3 * k)
        f = torch.from_numpy(W.load_sine(d, n)).cuda()
        reqs.append((d, n, P.Eps(fld), f))
    return reqs


def alone(ctx, reqs, **kw):
    out = []
    for d, n, eps, f in reqs:
        u, rep = P.solve(ctx, d, n, eps, f, **kw)
        assert rep["status"] == P.OK
        out.append((u.clone(), rep["cycles"]))
    return out


@pytest.mark.parametrize("precision", [P.MIXED, P.FP64])
def test_mix_equals_alone_deterministic(ctx, precision):
    kw = dict(BASE, precision=precision, publish=P.PUBLISH_DETERMINISTIC)
    reqs = make_requests(SHAPES)
    ref = alone(ctx, reqs, **kw)
    res = serving.replay(ctx, reqs, None, max_slots=4, keep=True, **kw)
    assert (res["status"] == P.OK).all()
    for i, (u, cyc) in enumerate(ref):
        assert res["cycles"][i] == cyc, i
        assert torch.equal(res["solutions"][i], u), i


def test_mix_matches_alone_async(ctx):
    kw = dict(BASE, publish=P.PUBLISH_ASYNC)
    reqs = make_requests(SHAPES, seed0=100)
    ref = alone(ctx, reqs, **kw)
    arr = W.poisson_arrivals(len(reqs), 2000.0, 5)
    res = serving.replay(ctx, reqs, arr, max_slots=3, keep=True, **kw)
    assert (res["status"] == P.OK).all()
    for i, (u, _) in enumerate(ref):
        e = float(torch.linalg.norm(res["solutions"][i] - u) / torch.linalg.norm(u))
        assert e <= 1e-6, (i, e)


def test_mix_equals_alone_parked(ctx):
    """Provisional target 1: every request parks on its provisional operator
    until the final one is built (without blocking the server), then cycles
    from the zero guess: bitwise the same result alone and in the mix."""
    kw = dict(BASE, publish=P.PUBLISH_ASYNC, prov_tol=1.0)
    reqs = make_requests(SHAPES, seed0=300)
    ref = alone(ctx, reqs, **kw)
    res = serving.replay(ctx, reqs, None, max_slots=4, keep=True, **kw)
    assert (res["status"] == P.OK).all()
    for i, (u, cyc) in enumerate(ref):
        assert res["cycles"][i] == cyc, i
        assert torch.equal(res["solutions"][i], u), i


def test_budget_admission(ctx):
    kw = dict(BASE, publish=P.PUBLISH_DETERMINISTIC)
    shapes = [(2, 64), (2, 32), (2, 64)]
    reqs = make_requests(shapes, seed0=200)
    ref = alone(ctx, reqs, **kw)
    big = max(P.solve_footprint(d, n, precision=P.MIXED, transfer=P.BOXMG) for d, n in shapes)
    # room for one state at a time: solves run one after another, evicting
    res = serving.replay(ctx, reqs, None, max_slots=4, budget_bytes=big * 1.05, keep=True, **kw)
    assert (res["status"] == P.OK).all()
    for i, (u, _) in enumerate(ref):
        assert torch.equal(res["solutions"][i], u), i
    # a request larger than the whole budget is rejected, the others run
    small = P.solve_footprint(2, 32, precision=P.MIXED, transfer=P.BOXMG)
    res = serving.replay(ctx, reqs, None, max_slots=4, budget_bytes=small * 1.05, **kw)
    assert list(res["status"]) == [P.ENOMEM, P.OK, P.ENOMEM]


def test_state_reuse_and_stats(ctx):
    kw = dict(BASE, publish=P.PUBLISH_DETERMINISTIC)
    reqs = make_requests([(2, 32)] * 4, seed0=300)
    srv = P.Server(ctx, max_slots=2, budget_bytes=1e10)
    try:
        us = []
        for d, n, eps, f in reqs:
            u = torch.zeros_like(f)
            srv.submit(d, n, eps, f, u, **kw)
            us.append(u)
        done = 0
        while done < len(reqs):
            fin, _, _ = srv.poll()
            done += fin
        st = srv.stats()
        assert st["completed"] == 4
        assert st["idle_states"] == 2  # two slots, each state reused by later requests
        one = P.solve_footprint(2, 32, precision=P.MIXED, transfer=P.BOXMG)
        assert st["resident_bytes"] <= 2 * one
    finally:
        srv.close()


def test_server_invalid(ctx):
    with pytest.raises(P.MgdError):
        P.Server(ctx, max_slots=0)
    srv = P.Server(ctx, max_slots=1)
    try:
        f = torch.zeros(33 * 33, dtype=torch.float64, device="cuda")
        u = torch.zeros_like(f)
        with pytest.raises(P.MgdError):
            srv.submit(2, 32, P.Eps(W.const_field(3)), f, u, **BASE)  # dimension mismatch
        with pytest.raises(P.MgdError):
            srv.result(12345)
    finally:
        srv.close()


def test_fresh_states_under_concurrency(ctx):
    """Many solves admitted at once on a new server, each on a newly created
    device state (its buffers cleared at creation must not race with the
    concurrent solve streams): every result matches its lone solve."""
    shapes = [(2, 128), (2, 256), (3, 24), (2, 192), (3, 32), (2, 128), (2, 256), (3, 16),
              (2, 64), (3, 24), (2, 256), (2, 96)]
    reqs = make_requests(shapes, seed0=400)
    kw = dict(BASE, schedule=P.UPFRONT)
    ref = alone(ctx, reqs, **kw)
    for _ in range(2):
        res = serving.replay(ctx, reqs, None, max_slots=8, keep=True, **kw)
        assert (res["status"] == P.OK).all(), res["status"]
        for i, (u, _) in enumerate(ref):
            assert torch.equal(res["solutions"][i], u), i
