"""lsq_fused_pass_noalloc (the allocation-free fused pass: partials in a static device array) against
lsq_fused_pass through the C ABI, on two calls in a row, the second with a smaller input (the array keeps
the first call's contents, which must not leak into the second).  With the same workgroup count (2 per
CU, below the array's cap) both take the same fixed-order reductions and must agree bit for bit; with
the default count (capped by the array at d = 1024) the results must meet the fused pass's own
summation bound against the FP64 reference A^T (A v)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(ctx, n, d, dtype, seed):
    import torch
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, d))
    if dtype == "f32":
        A = A.astype(np.float32)
    v, y = rng.standard_normal(d), rng.standard_normal(n)
    return A, torch.from_numpy(A).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(v).cuda(), v, y


@pytest.mark.parametrize("gpc", [2, 8])
def test_noalloc_fused_pass_matches(gpc):
    import torch

    from paper_1911_02675_amd import lsq
    lsq.tune("fused_groups_per_cu", gpc)
    try:
        with lsq.Context() as ctx:
            for n, d, dtype, seed in [(1 << 20, 1024, "f64", 1), (3001, 70, "f32", 2)]:
                say("noalloc", gpc, n, d, dtype)
                A, tA, ty, tv, v, y = _case(ctx, n, d, dtype, seed)
                Ad = A.astype(np.float64)
                for mode in (0, 1):
                    for f32 in ((False, True) if dtype == "f32" else (False,)):
                        w0 = torch.empty(d, dtype=torch.float64, device="cuda")
                        s0 = torch.empty(1, dtype=torch.float64, device="cuda")
                        w1 = torch.full((d,), np.nan, dtype=torch.float64, device="cuda")
                        s1 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
                        ctx.fused_pass(tA, ty, tv, w0, s0, mode=mode, f32_math=f32)
                        ctx.fused_pass_noalloc(tA, ty, tv, w1, s1, mode=mode, f32_math=f32)
                        torch.cuda.synchronize()
                        g0, g1 = w0.cpu().numpy(), w1.cpu().numpy()
                        q = Ad @ v if mode == 0 else y - Ad @ v
                        absq = np.abs(Ad) @ np.abs(v) + (0 if mode == 0 else np.abs(y))
                        u = 2.0 ** -24 if f32 else EPS
                        bound = 8 * (d + n) * u * (np.abs(Ad).T @ absq) + 1e-300
                        assert np.all(np.abs(g1 - Ad.T @ q) <= bound), (mode, f32)
                        assert abs(s1.item() - q @ q) <= 8 * (d + n) * u * (absq @ absq)
                        if gpc == 2 or n < 1 << 16:
                            # same grid as lsq_fused_pass: the same sums in the same order
                            assert np.array_equal(g0, g1) and s0.item() == s1.item(), (mode, f32)
                y0 = torch.zeros(n, dtype=torch.float64, device="cuda")
                with pytest.raises(lsq.LsqError) as e:
                    ctx.fused_pass_noalloc(tA, y0, tv, w1, s1, mode=2)
                assert e.value.status == lsq.LSQ_ERR_UNSUPPORTED
    finally:
        lsq.tune("fused_groups_per_cu", 8)
