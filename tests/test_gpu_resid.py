"""The double-double refinement residual (lsq_fused_pass mode 2) against the exact residual in rational
arithmetic, and the mixed form's refinement beyond the FP64 conditioning floor.

Bound for mode 2: every partial is a double-double with relative error O(u^2) of the sum of |q_j a_j|,
then one rounding, so |r - r_exact| <= 2u |r_exact| + 64 n u^2 sum_j |q_j a_j|.  Plain FP64 (mode 1)
is only good to about n u sum_j |q_j a_j|, which near the solution is far larger than |r|."""
import sys
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_02675_amd import lsq
    c = lsq.Context()
    yield c
    c.close()


# odd n (a padding row in the last pair), the vector and scalar column paths of both storage types, one
# chunk and several, and enough rows that wavefronts take several pairs (the prefetched path)
@pytest.mark.parametrize("n,d,f32", [(300, 8, True), (257, 7, True), (300, 6, False), (130, 130, True),
                                     (301, 12, False), (20001, 16, True), (4099, 64, False)])
def test_resid_dd_exact(ctx, n, d, f32):
    import torch
    rng = np.random.default_rng(n + d)
    A = rng.standard_normal((n, d))
    if f32:
        A = A.astype(np.float32).astype(np.float64)
    x = rng.standard_normal(d)
    # y close to A x: the residual is a small difference of large terms
    y = A @ x + 1e-9 * rng.standard_normal(n)
    Af = [[Fraction(v) for v in row] for row in A]
    xf = [Fraction(v) for v in x]
    q = [Fraction(y[j]) - sum(Af[j][k] * xf[k] for k in range(d)) for j in range(n)]
    r_exact = np.array([float(sum(q[j] * Af[j][e] for j in range(n))) for e in range(d)])
    absum = np.array([float(sum(abs(q[j] * Af[j][e]) for j in range(n))) for e in range(d)])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Ad = dev(A.astype(np.float32)) if f32 else dev(A)
    w = torch.empty(d, dtype=torch.float64, device="cuda")
    sc = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.fused_pass(Ad, dev(y), dev(x), w, sc, mode=2)
    torch.cuda.synchronize()
    got = w.cpu().numpy()
    err = np.abs(got - r_exact)
    bound = 2 * U * np.abs(r_exact) + 64 * n * U * U * absum
    say("  mode 2: max err / bound", float(np.max(err / bound)))
    assert np.all(err <= bound)
    # the plain FP64 pass is far less accurate here (the reason for mode 2)
    ctx.fused_pass(Ad, dev(y), dev(x), w, sc, mode=1)
    torch.cuda.synchronize()
    err1 = np.max(np.abs(w.cpu().numpy() - r_exact) / np.abs(r_exact))
    say("  mode 1: max relative error", float(err1))
    assert float(sc.cpu().numpy()[0]) > 0


def test_mixed_refinement_beyond_fp64_floor(ctx):
    """At kappa = 1e8 plain FP64 PCG stops at the conditioning floor; the refinement with the
    double-double residual reaches 1e-10 against the exact planted minimiser."""
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted
    n, d, m = 1 << 16, 128, 1024
    P = make_planted(n, d, 1e8, sigma=0.01, seed=91, want64=True, want32=True)
    A32 = torch.from_numpy(P["A32"]).cuda()
    y32 = torch.from_numpy(P["y32"]).cuda()
    xs = torch.from_numpy(P["x_star"]).cuda()
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    st, info = ctx.pcg_solve(A32, y32, lsq.sketch_desc("srht", m, seed=4, compute="f32"), x, tol=1e-10,
                             max_iter=300, mixed=1, max_refine=10, raise_on_error=False)
    Ad = A32.double()
    e = float(torch.linalg.norm(Ad @ (x - xs)) / torch.linalg.norm(Ad @ xs))
    say("  kappa 1e8 mixed: status", st, "refinements", info.refinements, "e_A", e)
    assert st == lsq.LSQ_OK
    assert e <= 1e-10


def test_mixed_refinement_from_nonzero_start(ctx):
    """A nonzero starting point takes the double-double residual from the first step (from x_0 = 0 the
    first residual is A^T y, taken by a plain pass); both starts reach the tolerance."""
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted
    n, d, m = 1 << 15, 96, 768
    P = make_planted(n, d, 1e6, sigma=0.01, seed=92, want64=True, want32=True)
    A32 = torch.from_numpy(P["A32"]).cuda()
    y32 = torch.from_numpy(P["y32"]).cuda()
    xs = torch.from_numpy(P["x_star"]).cuda()
    Ad = A32.double()
    ax = float(torch.linalg.norm(Ad @ xs))
    for x0 in (torch.zeros(d, dtype=torch.float64, device="cuda"), 0.5 * xs.clone()):
        x = x0.clone()
        st, info = ctx.pcg_solve(A32, y32, lsq.sketch_desc("srht", m, seed=5, compute="f32"), x, tol=1e-10,
                                 max_iter=300, mixed=1, max_refine=10, raise_on_error=False)
        e = float(torch.linalg.norm(Ad @ (x - xs))) / ax
        say("  start", "zero" if float(x0.abs().max()) == 0 else "0.5 x*", "status", st, "refinements",
            info.refinements, "iters", info.iters, "e_A", e)
        assert st == lsq.LSQ_OK
        assert e <= 1e-10


def test_mixed_fp32_transform_upgrade_at_kappa_1e8(ctx):
    """The precision form with an FP32 SRHT at kappa = 1e8: the FP32 transform's rounding weakens the
    preconditioner, the factor's diagonal spread (about kappa / 25) exceeds 1e6, and the solve retakes the
    sketch with an FP64 transform (lsq_set_option "sketch_upgrade", on by default).  Both settings reach the
    tolerance; the upgraded one needs fewer PCG iterations."""
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted
    n, d, m = 1 << 16, 128, 1024
    P = make_planted(n, d, 1e8, sigma=0.01, seed=94, want64=False, want32=True)
    A32 = torch.from_numpy(P["A32"]).cuda()
    y32 = torch.from_numpy(P["y32"]).cuda()
    xs = torch.from_numpy(P["x_star"]).cuda()
    Ad = A32.double()
    res = {}
    try:
        for up in (0, 1):
            ctx.set_option("sketch_upgrade", up)
            x = torch.zeros(d, dtype=torch.float64, device="cuda")
            st, info = ctx.pcg_solve(A32, y32, lsq.sketch_desc("srht", m, seed=4, compute="f32"), x, tol=1e-10,
                                     max_iter=300, mixed=1, max_refine=10, raise_on_error=False)
            e = float(torch.linalg.norm(Ad @ (x - xs)) / torch.linalg.norm(Ad @ xs))
            say("  sketch_upgrade", up, "status", st, "iters", info.iters, "e_A", e)
            assert st == lsq.LSQ_OK and e <= 1e-10
            res[up] = info.iters
    finally:
        ctx.set_option("sketch_upgrade", 1)
    assert res[1] < res[0]
