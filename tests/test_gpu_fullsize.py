"""Parity at the full benchmark size (n = 2^22, d = 1024, kappa = 1e6, m = 4096), in the launch
configuration bench.py times (the autotuner's table applied), on outputs the oracle can compute one
by one and on properties that hold at any size:

  * sampled rows of S A (SRHT in FP64 and FP32, Gaussian in FP64 and BF16), each recomputed by the
    oracle directly from its definition (a signed sum over all n rows of A for one output row,
    on a sample of columns), within summation-order bounds of the arithmetic;
  * the FP64 and mixed solves against the exact minimiser of the planted problem (relative A-norm
    error 1e-10); the normal-equation residual ||A^T (y - A x)|| / ||A^T y||, which the A-norm error
    bounds by kappa times, is reported and checked at that level."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_ROWS, D, M, KAPPA, SEED = 1 << 22, 1024, 4096, 1e6, 3001
EPS64, EPS32 = 2.0 ** -52, 2.0 ** -23


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big():
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted
    say("full size: generating the planted problem")
    P = make_planted(N_ROWS, D, KAPPA, sigma=0.01, seed=SEED, want64=True, want32=True)
    ctx = lsq.Context()
    out = dict(P=P, ctx=ctx, A64=torch.from_numpy(P["A64"]).cuda(), y64=torch.from_numpy(P["y64"]).cuda(),
               A32=torch.from_numpy(P["A32"]).cuda(), y32=torch.from_numpy(P["y32"]).cuda(),
               xs=torch.from_numpy(P["x_star"]).cuda())
    torch.cuda.synchronize()
    yield out
    ctx.close()


def _sketch(big, A, y, desc, m=M):
    import torch
    SA = torch.zeros((m, D), dtype=torch.float64, device="cuda")
    big["ctx"].sketch(A, y, desc, SA)
    torch.cuda.synchronize()
    return SA.cpu().numpy()


COLS = np.arange(0, D, 16)  # 64 sampled columns
ROWS = [0, 1, 2047, 4095]


@pytest.mark.parametrize("compute,m", [("f64", M), ("f32", M), ("f32", 6 * M), ("f64", 6 * M)])
def test_fullsize_srht_rows(big, compute, m):
    """m = 4096 and the chooser's 24d (buckets of about 96 selected rows: the folded pass B)."""
    from oracle.draws import padded_length, srht_rows, srht_signs
    from oracle.sketch import hadamard_entry, srht_sketch_rows
    from paper_1911_02675_amd import lsq
    A = big["P"]["A64"] if compute == "f64" else big["P"]["A32"].astype(np.float64)
    Ad, yd = (big["A64"], big["y64"]) if compute == "f64" else (big["A32"], big["y32"])
    rows = [0, 1, m // 2 - 1, m - 1]
    got = _sketch(big, Ad, yd, lsq.sketch_desc("srht", m, seed=SEED, compute=compute), m)[np.ix_(rows, COLS)]
    ref = srht_sketch_rows(A, m, SEED, 0, rows, cols=COLS)
    # any summation order of n signed terms: |error| <= (log2 N + 2) eps sum |a_j| / sqrt(m)
    absum = np.abs(A[:, COLS]).sum(axis=0)[None, :] / np.sqrt(m)
    eps = EPS64 if compute == "f64" else EPS32
    bound = (np.log2(padded_length(N_ROWS)) + 2) * eps * absum
    say(f"  SRHT {compute}: max err / bound {np.max(np.abs(got - ref) / bound):.3f}")
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("compute", ["f64", "bf16"])
def test_fullsize_gaussian_rows(big, compute):
    from oracle.draws import gaussian_normals, round_bf16
    from paper_1911_02675_amd import lsq
    A = big["P"]["A32"].astype(np.float64)
    got = _sketch(big, big["A32"], big["y32"], lsq.sketch_desc("gaussian", M, seed=SEED, compute=compute))
    rows = [0, 4095]
    j = np.arange(N_ROWS)
    for i in rows:
        g = gaussian_normals(SEED, 0, np.full(N_ROWS, i), j)
        if compute == "bf16":
            g = round_bf16(g)
        ref = (g @ A[:, COLS]) / np.sqrt(M)
        prod = (np.abs(g) @ np.abs(A[:, COLS])) / np.sqrt(M)
        maxterm = np.abs(g).max() * np.abs(A[:, COLS]).max(axis=0) / np.sqrt(M)
        if compute == "f64":
            # single-precision normals (<= 8e-6 absolute each) and FP64 sums
            bound = 8e-6 * (np.abs(A[:, COLS]).sum(axis=0) / np.sqrt(M)) + 64 * EPS64 * prod
        else:
            # FP32 chains of 256 rows folded into FP64, the three-term split, and a few BF16 rounding
            # flips of normals whose single- and double-precision values straddle a rounding boundary
            bound = 64 * 2.0 ** -24 * prod + 64 * 2.0 ** -7 * maxterm
        err = np.abs(got[i, COLS] - ref)
        say(f"  Gaussian {compute} row {i}: max err / bound {np.max(err / bound):.3f}")
        assert np.all(err <= bound)


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_fullsize_solve(big, form):
    import torch

    from paper_1911_02675_amd import autotune, lsq
    autotune.apply("f64" if form == "fp64" else "f32", D)
    try:
        x = torch.zeros(D, dtype=torch.float64, device="cuda")
        if form == "fp64":
            A, y = big["A64"], big["y64"]
            st, info = big["ctx"].pcg_solve(A, y, lsq.sketch_desc("srht", M, seed=SEED), x, tol=1e-10, max_iter=200)
        else:
            A, y = big["A32"], big["y32"]
            st, info = big["ctx"].pcg_solve(A, y, lsq.sketch_desc("srht", M, seed=SEED, compute="f32"), x,
                                            tol=1e-10, max_iter=200, mixed=1, max_refine=8)
        Ad = A.double() if form == "mixed" else A
        xs = big["xs"]
        e = float(torch.linalg.norm(Ad @ (x - xs)) / torch.linalg.norm(Ad @ xs))
        g = float(torch.linalg.norm(Ad.T @ (y - Ad @ x)) / torch.linalg.norm(Ad.T @ y))
        del Ad
        say(f"  {form}: iters {info.iters}, e_A {e:.2e}, normal-equation residual {g:.2e}")
        assert e <= 1e-10
        assert g <= KAPPA * 1e-10
    finally:
        lsq.tune("fused_groups_per_cu", 8)
