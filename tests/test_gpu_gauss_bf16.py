"""GPU parity of the Gaussian precision form (BF16 matrix cores, A split into three BF16 terms,
FP32 accumulation in short chains folded into FP64) against the oracle's BF16-rounded embedding.

Bound per entry (i, c) of S A: the three-term split and the FP32 chains contribute at most
c1 * 2^-24 * (|S_bf16| |A|)_ic; a normal whose single-precision Box-Muller value and the oracle's
double-precision value round to different BF16 neighbours (probability about 1e-4 per entry) moves
one term by one BF16 step, at most 2^-7 * max_j |S_ij A_jc| each; a few such flips are allowed."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_02675_amd import lsq
    c = lsq.Context()
    yield c
    c.close()


# (n, d, m, dtype, rows per chunk of the planes form or None).  d >= 384 takes the planes form (the three
# BF16 terms of A formed once per chunk of rows, 64 x 512 output tiles); ragged n, d and m, FP64 A,
# several chunks (a small chunk size), and an m that leaves k-splits empty in the last chunk.
CASES = [(5000, 33, 100, "f32", None), (5000, 300, 300, "f64", None), (70000, 64, 200, "f32", None),
         (3000, 1, 17, "f32", None), (20001, 257, 129, "f32", None),
         (20001, 700, 130, "f32", None), (9000, 512, 64, "f64", None), (5000, 384, 300, "f32", None),
         (40000, 520, 70, "f32", 4096), (6000, 1000, 33, "f32", 2048)]
# planes form edge cases (n >= d): a ragged last 32-row step with m below one row tile, a single row of
# S, the largest d, and rows of A at a stride wider than d (FP32 and FP64)
EDGE = [(401, 384, 3, "f32", 0), (600, 512, 1, "f32", 0), (1100, 1024, 130, "f32", 0), (3000, 400, 65, "f32", 5),
        (2000, 600, 40, "f64", 3)]


@pytest.mark.parametrize("n,d,m,dtype,chunk", CASES)
def test_gauss_bf16_sketch(ctx, n, d, m, dtype, chunk):
    from paper_1911_02675_amd import lsq
    say("gauss bf16", n, d, m, dtype, chunk)
    try:
        if chunk:
            lsq.tune("gauss_chunk_rows", chunk)
        _check_bf16_sketch(ctx, n, d, m, dtype)
    finally:
        lsq.tune("gauss_chunk_rows", 0)


@pytest.mark.parametrize("n,d,m,dtype,pad", EDGE)
def test_gauss_bf16_planes_edges(ctx, n, d, m, dtype, pad):
    say("gauss bf16 planes edge", n, d, m, dtype, pad)
    _check_bf16_sketch(ctx, n, d, m, dtype, pad)


def test_gauss_bf16_both_forms(ctx):
    """At d >= 384 the tile form (forced by a high threshold) and the planes form both meet the bound."""
    from paper_1911_02675_amd import lsq
    try:
        lsq.tune("gauss_planes_min_d", 1 << 20)
        _check_bf16_sketch(ctx, 20001, 700, 130, "f32")
    finally:
        lsq.tune("gauss_planes_min_d", 384)


def _check_bf16_sketch(ctx, n, d, m, dtype, pad=0):
    import torch

    from oracle.draws import gaussian_normals, round_bf16
    from oracle.sketch import gaussian_sketch_bf16
    from paper_1911_02675_amd import lsq
    rng = np.random.default_rng(n + d)
    A = rng.standard_normal((n, d)) * rng.uniform(0.5, 2.0, d)[None, :]
    if dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
    Ah = A.astype(np.float32) if dtype == "f32" else A
    if pad:
        # rows at a stride of d + pad elements: a view of a wider matrix
        W = np.zeros((n, d + pad), dtype=Ah.dtype)
        W[:, :d] = Ah
        Ad = torch.from_numpy(W).cuda()[:, :d]
    else:
        Ad = torch.from_numpy(Ah).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    SA = torch.zeros((m, d), dtype=torch.float64, device="cuda")
    seed = 31 + n
    ctx.sketch(Ad, y, lsq.sketch_desc("gaussian", m, seed=seed, compute="bf16"), SA)
    torch.cuda.synchronize()
    got = SA.cpu().numpy()
    ref = gaussian_sketch_bf16(A, m, seed)
    Sb = round_bf16(gaussian_normals(seed, 0, np.arange(m)[:, None], np.arange(n)[None, :])) / np.sqrt(m)
    absprod = np.abs(Sb) @ np.abs(A)
    maxterm = np.max(np.abs(Sb)[:, :, None] * np.abs(A)[None, :, :], axis=1) if n * m * d <= 2e8 else None
    err = np.abs(got - ref)
    if maxterm is None:
        maxterm = np.abs(Sb).max(axis=1)[:, None] * np.abs(A).max(axis=0)[None, :]
    bound = 64 * 2.0 ** -24 * absprod + 4 * 2.0 ** -7 * maxterm
    say(f"  max err / bound {np.max(err / bound):.3f}, max rel to |S||A| {np.max(err / absprod):.2e}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("d", [128, 512])
def test_gauss_bf16_preconditioner_quality(ctx, d):
    """The BF16 sketch is a working preconditioner at kappa = 1e6: PCG to 1e-10 in about the
    iterations of the FP64 Gaussian sketch with the same draws (tile form at d = 128, planes form at
    d = 512)."""
    import torch

    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_planted
    P = make_planted(1 << 15, d, 1e6, sigma=0.01, seed=77, want64=False, want32=True)
    A32, y, xs = P["A32"], P["y32"], P["x_star"]
    Ad, yd = torch.from_numpy(A32).cuda(), torch.from_numpy(y).cuda()
    its = {}
    for comp in ("f64", "bf16"):
        x = torch.zeros(d, dtype=torch.float64, device="cuda")
        st, info = ctx.pcg_solve(Ad, yd, lsq.sketch_desc("gaussian", 4 * d, seed=5, compute=comp), x, tol=1e-10,
                                 mixed=1, max_refine=10, max_iter=300)
        torch.cuda.synchronize()
        e = a_norm_error(A32.astype(np.float64), x.cpu().numpy(), xs)
        its[comp] = info.iters
        say(f"  {comp}: iters {info.iters}, e_A {e:.2e}")
        assert e <= 1e-10
    assert its["bf16"] <= its["f64"] + 3
