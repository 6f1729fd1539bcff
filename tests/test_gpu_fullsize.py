"""Parity at the full benchmark size (n = 2^22, d = 1024, kappa = 1e6), in the launch configuration
bench.py times (the autotuner's table applied; the sketch size m = 65536 that the Section 6 chooser
picks for both forms, and m = 4096 = 4d), on outputs the oracle can compute one by one and on
properties that hold at any size:

  * sampled rows of S A (SRHT in FP64 and FP32, Gaussian in FP64 and BF16), each recomputed by the
    oracle directly from its definition (a signed sum over all n rows of A for one output row,
    on a sample of columns), within summation-order bounds of the arithmetic;
  * exact SRHT parity: with integer A in {-3..3} every partial sum of the transform is an integer below
    3 N = 1.26e7 < 2^24, so the FP32 and FP64 paths (pass A, the 4- and 8-point folds, the matrix-core
    chains) must reproduce the oracle's integer sums exactly: 64 output rows from 64 distinct k_lo
    buckets, all 1024 columns, at m = 65536 (the streamed 16-point forms), 40960 (the staged 8-point
    forms) and 24576;
  * the FP64 and mixed solves against the exact minimiser of the planted problem (relative A-norm
    error 1e-10) at m = 4096 and 65536; the normal-equation residual ||A^T (y - A x)|| / ||A^T y||,
    which the A-norm error bounds by kappa times, is reported and checked at that level;
  * the mixed solve at kappa = 1e8 (beyond the FP64 conditioning floor of plain PCG) to 1e-10."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_ROWS, D, M, KAPPA, SEED = 1 << 22, 1024, 4096, 1e6, 3001
M_BENCH = 65536
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
            # FP64 normals within a few ulp of the oracle's and FP64 sums in any order
            bound = 80 * EPS64 * prod
        else:
            # FP32 chains of 256 rows folded into FP64, the three-term split, and a few BF16 rounding
            # flips of normals whose single- and double-precision values straddle a rounding boundary
            bound = 64 * 2.0 ** -24 * prod + 64 * 2.0 ** -7 * maxterm
        err = np.abs(got[i, COLS] - ref)
        say(f"  Gaussian {compute} row {i}: max err / bound {np.max(err / bound):.3f}")
        assert np.all(err <= bound)


@pytest.mark.parametrize("m", [M, M_BENCH])
@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_fullsize_solve(big, form, m):
    import torch

    from paper_1911_02675_amd import autotune, lsq
    autotune.apply("f64" if form == "fp64" else "f32", D)
    try:
        x = torch.zeros(D, dtype=torch.float64, device="cuda")
        if form == "fp64":
            A, y = big["A64"], big["y64"]
            st, info = big["ctx"].pcg_solve(A, y, lsq.sketch_desc("srht", m, seed=SEED), x, tol=1e-10, max_iter=200)
        else:
            A, y = big["A32"], big["y32"]
            st, info = big["ctx"].pcg_solve(A, y, lsq.sketch_desc("srht", m, seed=SEED, compute="f32"), x,
                                            tol=1e-10, max_iter=200, mixed=1, max_refine=8)
        Ad = A.double() if form == "mixed" else A
        xs = big["xs"]
        e = float(torch.linalg.norm(Ad @ (x - xs)) / torch.linalg.norm(Ad @ xs))
        g = float(torch.linalg.norm(Ad.T @ (y - Ad @ x)) / torch.linalg.norm(Ad.T @ y))
        del Ad
        say(f"  {form} m={m}: status {st}, iters {info.iters}, e_A {e:.2e}, normal-equation residual {g:.2e}")
        assert st == 0
        assert e <= 1e-10
        assert g <= KAPPA * 1e-10
    finally:
        lsq.tune("fused_groups_per_cu", 8)


@pytest.fixture(scope="module")
def intA():
    import torch

    from synth import make_integer_matrix
    say("full size: generating the integer matrix")
    Ai = make_integer_matrix(N_ROWS, D, 3, seed=SEED)
    yield Ai, torch.from_numpy(Ai).cuda()


def _distinct_bucket_rows(m, count=64):
    """Output positions spread over [0, m) whose selected rows k lie in distinct k_lo = k mod 256
    buckets (first and last position included)."""
    from oracle.draws import padded_length, srht_rows
    k = srht_rows(SEED, 0, padded_length(N_ROWS), m)
    out, seen = [], set()
    for pos in list(np.linspace(0, m - 1, 4 * count).astype(int)) + [m - 1]:
        if int(k[pos]) % 256 not in seen:
            seen.add(int(k[pos]) % 256)
            out.append(int(pos))
    if m - 1 not in out:
        out[-1] = m - 1
    return sorted(out[:count])


_EXACT_REF = {}


@pytest.mark.parametrize("m", [M_BENCH, 40960, 24576])
@pytest.mark.parametrize("compute", ["f32", "f64"])
def test_fullsize_srht_exact(big, intA, compute, m):
    """Integer A: the GPU S A times sqrt(m) must be the oracle's integer sums exactly."""
    import torch

    from oracle.sketch import srht_sketch_rows
    from paper_1911_02675_amd import lsq
    Ai, At = intA
    which = _distinct_bucket_rows(m)
    assert len(which) == 64
    Ad = At.to(torch.float32 if compute == "f32" else torch.float64)
    y0 = torch.zeros(N_ROWS, dtype=torch.float64, device="cuda")
    got = _sketch(big, Ad, y0, lsq.sketch_desc("srht", m, seed=SEED, compute=compute), m)[which]
    del Ad
    if m not in _EXACT_REF:
        say(f"  oracle: 64 rows x {D} columns of S A at m={m}")
        _EXACT_REF[m] = srht_sketch_rows(Ai, m, SEED, 0, which)
    ref = _EXACT_REF[m]
    gi, ri = got * np.sqrt(m), ref * np.sqrt(m)
    assert np.max(np.abs(ri - np.rint(ri))) < 1e-6  # the oracle's sums are integers
    nbad = int(np.sum(np.rint(gi) != np.rint(ri)))
    say(f"  SRHT {compute} m={m}: {nbad} of {gi.size} entries differ; max |gpu - oracle| / ulp "
        f"{np.max(np.abs(got - ref) / np.spacing(np.maximum(np.abs(ref), 1e-300))):.2f}")
    assert nbad == 0
    # each side rounds once when scaling by 1/sqrt(m): at most 2 ulp apart
    assert np.all(np.abs(got - ref) <= 2 * np.spacing(np.abs(ref)))


def test_fullsize_mixed_kappa_1e8(big):
    """Mixed form at kappa = 1e8, m = 65536: the refinement residual in double-double arithmetic takes
    the solve to the exact minimiser of the stored FP32 problem below 1e-10."""
    import torch

    from paper_1911_02675_amd import autotune, lsq
    from synth import make_planted
    say("full size: generating the kappa = 1e8 planted problem (FP32)")
    P = make_planted(N_ROWS, D, 1e8, sigma=0.01, seed=SEED + 8, want64=False, want32=True)
    A, y = torch.from_numpy(P["A32"]).cuda(), torch.from_numpy(P["y32"]).cuda()
    xs = torch.from_numpy(P["x_star"]).cuda()
    del P
    autotune.apply("f32", D)
    try:
        x = torch.zeros(D, dtype=torch.float64, device="cuda")
        st, info = big["ctx"].pcg_solve(A, y, lsq.sketch_desc("srht", M_BENCH, seed=SEED, compute="f32"), x,
                                        tol=1e-10, max_iter=200, mixed=1, max_refine=8)
        Ad = A.double()
        e = float(torch.linalg.norm(Ad @ (x - xs)) / torch.linalg.norm(Ad @ xs))
        del Ad
        say(f"  mixed kappa=1e8: status {st}, iters {info.iters}, refinements {info.refinements}, e_A {e:.2e}")
        assert st == 0
        assert e <= 1e-10
    finally:
        lsq.tune("fused_groups_per_cu", 8)
