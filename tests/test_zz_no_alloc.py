"""The allocation-free compression (static device scratch) against the
allocating entry point: the same store byte for byte, on two calls in a row
on one device with the second smaller (the scratch keeps the first call's
contents, which the second must not see)."""
import numpy as np
import pytest
import torch

P = pytest.importorskip("paper_2005_03606_amd")
import workload as W  # noqa: E402


def _level(ctx, d, n, seed):
    fld = W.balls_field(d, 12, seed, r_lo=0.05, r_hi=0.3, eps_in=1e3)
    eps = P.Eps(fld)
    K, _, _ = P.assemble_cells(ctx, d, n, 4, eps, P.MIXED)
    S32 = P.gather_stencils(ctx, d, n, K, P.MIXED, P.MIXED)
    return S32, P.centre_samples(ctx, d, n, eps)


def _store(ctx, d, n, S32, eps_c, noalloc, policy):
    h = P.Hierarchy(ctx, d, n, precision=P.MIXED, transfer=P.BOXMG)
    if noalloc:
        h.compress_noalloc(S32, eps_c, *policy)
    else:
        h.compress(S32, eps_c, *policy)
    tt, off, pay = h.store_export()
    out = [t.cpu().numpy().copy() for t in (tt, off, pay)] + [h.level_stencils(0).cpu().numpy()]
    tiers = h.store_info()[2]
    h.close()
    return out, tiers


@pytest.mark.gpu
@pytest.mark.parametrize("d,sizes", [(3, (40, 16)), (2, (256, 96))])
def test_compress_noalloc_equals_compress(d, sizes):
    """Per size, every tier forced in turn (FP8, FP16, FP32) and the dynamic
    choice; the second size is the smaller one."""
    ctx = P.Context(0)
    for n in sizes:
        S32, eps_c = _level(ctx, d, n, 7 + n)
        for policy in ((1, 1, 0.0, 0.0), (2, 2, 0.0, 0.0), (3, 3, 0.0, 0.0), (1, 3, 0.0, 1e-4)):
            ref, tiers = _store(ctx, d, n, S32, eps_c, False, policy)
            got, tiers2 = _store(ctx, d, n, S32, eps_c, True, policy)
            assert tiers == tiers2
            if policy[0] == policy[1]:
                assert tiers[policy[0]] > 0, (policy, tiers)
            for a, b in zip(ref, got):
                assert a.shape == b.shape and np.array_equal(a, b)
    ctx.close()


@pytest.mark.gpu
def test_compress_noalloc_rejects_levels_beyond_its_scratch():
    ctx = P.Context(0)
    d, n = 3, 128  # 129^3 vertices x 53 bytes > 64 MiB
    h = P.Hierarchy(ctx, d, n, precision=P.MIXED)
    S32 = torch.zeros(13 * (n + 1) ** 3, dtype=torch.float32, device="cuda")
    eps_c = torch.ones(n ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(P.MgdError) as e:
        h.compress_noalloc(S32, eps_c, 2, 2, 0.0, 0.0)
    assert e.value.code == P.EINVAL and "at most" in str(e.value)
    h.close()
    ctx.close()
