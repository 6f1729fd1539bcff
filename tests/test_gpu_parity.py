"""GPU parity: the HIP library (through its C ABI) against the CPU oracle, element by element, on
seeded inputs at sizes the oracle finishes in seconds, spanning several tiles and ragged tails.

Tolerances come from the arithmetic: integer draws are bit-exact; floating-point results are
compared against bounds of the form c * eps * (|S| |A|) that any summation order satisfies; solves
against the relative A-norm error 1e-10 (or, where FP64 conditioning limits every solver, four
times the disagreement of two backward-stable FP64 solvers on the same input)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_02675_amd import lsq
    c = lsq.Context()
    yield c
    c.close()


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ----------------------------------------------------------------------------------------------
# draws: bit-exact
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("N,m,seed,t", [(8, 8, 1, 0), (4096, 256, 7, 0), (1 << 16, 1000, 3, 5),
                                        (1 << 20, 4096, 11, 2)])
def test_srht_draws_bit_exact(ctx, N, m, seed, t):
    from oracle import draws
    torch = _torch()
    say("srht draws", N, m, seed, t)
    signs = torch.empty(N, dtype=torch.int8, device="cuda")
    rows = torch.empty(m, dtype=torch.int64, device="cuda")
    ctx.draw_srht(seed, t, N, m, signs, rows)
    assert np.array_equal(host(signs).astype(np.float64), draws.srht_signs(seed, t, N))
    assert np.array_equal(host(rows), draws.srht_rows(seed, t, N, m))


@pytest.mark.parametrize("n,m,s,seed,t", [(1, 1, 1, 0, 0), (5000, 64, 4, 3, 1), (30000, 1024, 8, 9, 0),
                                          (777, 16, 16, 2, 3), (4096, 3, 2, 5, 0)])
def test_sjlt_draws_bit_exact(ctx, n, m, s, seed, t):
    from oracle import draws
    torch = _torch()
    say("sjlt draws", n, m, s)
    tg = torch.empty(n * s, dtype=torch.int32, device="cuda")
    sg = torch.empty(n * s, dtype=torch.int8, device="cuda")
    ctx.draw_sjlt(seed, t, n, m, s, tg, sg)
    otg, osg = draws.sjlt_draws(seed, t, n, m, s)
    assert np.array_equal(host(tg).reshape(n, s), otg)
    assert np.array_equal(host(sg).reshape(n, s).astype(np.float64), osg)


def test_gaussian_draws_close(ctx):
    from oracle import draws
    torch = _torch()
    m, j0, nc = 37, 5, 1003
    say("gaussian draws")
    G = torch.empty((m, nc), dtype=torch.float64, device="cuda")
    ctx.draw_gaussian(123, 4, m, j0, nc, G)
    ref = draws.gaussian_normals(123, 4, np.arange(m)[:, None], np.arange(j0, j0 + nc)[None, :])
    # FP64 Box-Muller on both sides from the same exact u1, u2 and the same rounded angle: the device
    # library's log, sqrt and sincos against numpy's, a few ulp of each value
    ulps = np.abs(host(G) - ref) / np.spacing(np.abs(ref))
    say("  max ulp", ulps.max(), "99.9th percentile", np.percentile(ulps, 99.9))
    assert ulps.max() <= 4.0, ulps.max()


# ----------------------------------------------------------------------------------------------
# fused pass
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,d", [(1, 1), (777, 7), (1000, 33), (3001, 64), (2500, 100), (4099, 512),
                                 (2049, 1024), (1100, 1023)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_pass(ctx, n, d, dtype):
    torch = _torch()
    say("fused", n, d, dtype)
    rng = np.random.default_rng(n * 7 + d)
    A = rng.standard_normal((n, d))
    if dtype == "f32":
        A = A.astype(np.float32)
    Ad = A.astype(np.float64)
    v = rng.standard_normal(d)
    y = rng.standard_normal(n)
    tA, ty, tv = dev(A), dev(y), dev(v)
    w = torch.empty(d, dtype=torch.float64, device="cuda")
    sc = torch.empty(1, dtype=torch.float64, device="cuda")
    for mode in (0, 1):
        ctx.fused_pass(tA, ty, tv, w, sc, mode=mode)
        q = Ad @ v if mode == 0 else y - Ad @ v
        wr = Ad.T @ q
        bound = (np.abs(Ad).T @ (np.abs(Ad) @ np.abs(v) + (0 if mode == 0 else np.abs(y))))
        tol = 4 * (d + n) * EPS * bound + 1e-300
        assert np.all(np.abs(host(w) - wr) <= tol)
        assert abs(host(sc)[0] - q @ q) <= 4 * (d + n) * EPS * ((np.abs(Ad) @ np.abs(v) + (mode * np.abs(y))) ** 2).sum()
    if dtype == "f32":
        ctx.fused_pass(tA, ty, tv, w, sc, mode=0, f32_math=True)
        wr = Ad.T @ (Ad @ v)
        bound = np.abs(Ad).T @ (np.abs(Ad) @ np.abs(v))
        assert np.all(np.abs(host(w) - wr) <= 8 * (d + n) * 2.0 ** -24 * bound + 1e-30)


# ----------------------------------------------------------------------------------------------
# sketches
# ----------------------------------------------------------------------------------------------
def _sa(ctx, A, kind, m, seed, t=0, s=1, compute="f64"):
    from paper_1911_02675_amd import lsq
    torch = _torch()
    n, d = A.shape
    SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
    desc = lsq.sketch_desc(kind, m, seed=seed, t=t, s=s, compute=compute)
    ctx.sketch(dev(A), dev(np.zeros(n)), desc, SA)
    return host(SA)


@pytest.mark.parametrize("n,d,m", [(100, 3, 16), (4096, 64, 256), (3000, 70, 300), (20000, 129, 700),
                                   (1 << 14, 256, 2048), (60000, 70, 8000), (1 << 15, 48, 12000),
                                   (1 << 17, 40, 8000), (200000, 33, 9000), (1 << 17, 20, 100000),
                                   (300000, 130, 20000), (1 << 17, 24, 40000)])
def test_srht_sketch(ctx, n, d, m):
    from oracle import draws, sketch
    say("srht sketch", n, d, m)
    A = np.random.default_rng(n + d).standard_normal((n, d))
    got = _sa(ctx, A, "srht", m, seed=17, t=1)
    ref = sketch.srht_sketch(A, m, 17, 1)
    N = draws.padded_length(n)
    scale = np.abs(A).sum(axis=0)[None, :] / math.sqrt(m)
    assert np.all(np.abs(got - ref) <= 8 * (math.log2(N) + 2) * EPS * scale)
    # FP32 transform: single-precision butterflies, same bound with eps_32
    A32 = A.astype(np.float32)
    got32 = _sa(ctx, A32, "srht", m, seed=17, t=1, compute="f32")
    ref32 = sketch.srht_sketch(A32.astype(np.float64), m, 17, 1)
    assert np.all(np.abs(got32 - ref32) <= 8 * (math.log2(N) + 2) * 2.0 ** -24 * scale)


@pytest.mark.parametrize("n,d,m", [(300000, 130, 20000), (1 << 17, 20, 100000)])
def test_srht_pass_b_forms(ctx, n, d, m):
    """The large-bucket forms of the sampled transform (option srht_passb: 0 automatic, 1
    register-direct for FP32 T, 2 eight wavefronts, 3 sixteen with the 4-point fold, 4 sixteen with the
    8-point fold, 5 and 6 the intermediate streamed into LDS with the 8- and 16-point folds) all meet the
    oracle bound; 2 and 3 take the same arithmetic per output element and agree bitwise, and so do the
    automatic form and the streamed 16-point form it picks at 390 rows per bucket."""
    from oracle import draws, sketch
    from paper_1911_02675_amd import lsq
    say("srht pass B forms", n, d, m)
    A = np.random.default_rng(n - d).standard_normal((n, d))
    N = draws.padded_length(n)
    scale = np.abs(A).sum(axis=0)[None, :] / math.sqrt(m)
    ref = sketch.srht_sketch(A, m, 9, 2)
    ref32 = sketch.srht_sketch(A.astype(np.float32).astype(np.float64), m, 9, 2)
    got = {}
    try:
        for mode in (0, 1, 2, 3, 4, 5, 6):
            ctx.set_option("srht_passb", mode)
            got[mode] = (_sa(ctx, A, "srht", m, seed=9, t=2),
                         _sa(ctx, A.astype(np.float32), "srht", m, seed=9, t=2, compute="f32"))
    finally:
        ctx.set_option("srht_passb", 0)
    for mode, (g64, g32) in got.items():
        assert np.all(np.abs(g64 - ref) <= 8 * (math.log2(N) + 2) * EPS * scale), mode
        assert np.all(np.abs(g32 - ref32) <= 8 * (math.log2(N) + 2) * 2.0 ** -24 * scale), mode
    assert np.array_equal(got[2][0], got[3][0]) and np.array_equal(got[2][1], got[3][1])
    # the automatic form at 390 rows per bucket is the streamed one with the 16-point fold
    if m / 256 >= 192:
        assert np.array_equal(got[0][0], got[6][0]) and np.array_equal(got[0][1], got[6][1])


@pytest.mark.parametrize("n,d,m", [(100, 3, 16), (4096, 64, 256), (20000, 129, 700), (1 << 15, 48, 12000),
                                   (300000, 130, 20000), (1 << 17, 20, 100000), (1 << 18, 64, 40000),
                                   (1 << 18, 24, 160000)])
def test_srht_exact_integer(ctx, n, d, m):
    """Exact parity of every SRHT form.  With A in {-2..2} every partial sum of the transform is an
    integer of magnitude at most 2 N < 2^24, exact in FP32 and FP64 alike, so S A sqrt(m) must equal
    the oracle's transform exactly: every pass B form (option srht_passb 0-6, each taken where the
    buckets are large), FP64 and FP32 A, FP64 and FP32 transforms, the 16-byte vector pass A and the
    scalar one (leading dimension d + 1).  A wrong sign, index or fold in any of them changes some
    output integer.  m = 100000 over 2^17 rows (390 per bucket) makes the streamed forms take two
    sweeps over some buckets' intermediate, m = 160000 (625 per bucket) two tile chunks."""
    from oracle import sketch
    from paper_1911_02675_amd import lsq
    torch = _torch()
    say("srht exact", n, d, m)
    Ai = np.random.default_rng(n + 3 * d).integers(-2, 3, size=(n, d)).astype(np.float64)
    ref = sketch.srht_sketch(Ai, m, 9, 2) * math.sqrt(m)
    assert np.max(np.abs(ref - np.rint(ref))) < 1e-6
    ref = np.rint(ref)
    pad = torch.zeros((n, d + 1), dtype=torch.float64, device="cuda")
    pad[:, :d] = dev(Ai)
    y0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    cases = {"f64/f64": (dev(Ai), "f64"), "f32/f32": (dev(Ai.astype(np.float32)), "f32"),
             "f32/f64": (dev(Ai.astype(np.float32)), "f64"), "f64/f32": (dev(Ai), "f32"),
             "f64 lda=d+1": (pad[:, :d], "f64"), "f32 lda=d+1": (pad.float()[:, :d], "f32")}
    modes = (0, 1, 2, 3, 4, 5, 6) if m > 24 * 256 else (0,)
    try:
        for mode in modes:
            ctx.set_option("srht_passb", mode)
            for name, (A, compute) in cases.items():
                SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
                ctx.sketch(A, y0, lsq.sketch_desc("srht", m, seed=9, t=2, compute=compute), SA)
                got = host(SA) * math.sqrt(m)
                bad = int(np.sum(np.rint(got) != ref))
                assert bad == 0, (mode, name, bad)
                assert np.max(np.abs(got - ref)) <= 4 * EPS * max(1.0, np.abs(ref).max()), (mode, name)
    finally:
        ctx.set_option("srht_passb", 0)


@pytest.mark.parametrize("n,d,m,s", [(100, 3, 16, 1), (5000, 64, 256, 4), (20001, 100, 512, 8),
                                     (9000, 257, 64, 2), (4096, 32, 4096, 1)])
def test_sjlt_sketch(ctx, n, d, m, s):
    from oracle import sketch
    say("sjlt sketch", n, d, m, s)
    A = np.random.default_rng(n + s).standard_normal((n, d))
    got = _sa(ctx, A, "sjlt", m, seed=5, t=3, s=s)
    ref = sketch.sjlt_sketch(A, m, s, 5, 3)
    S = sketch.sjlt_matrix(n, m, s, 5, 3) if n * m <= 5e7 else None
    bound = (np.abs(S) @ np.abs(A)) if S is not None else np.abs(A).sum(axis=0)[None, :]
    assert np.all(np.abs(got - ref) <= 4 * (n * s / m + 2) * EPS * bound + 1e-300)
    # deterministic: bitwise identical on a second run
    assert np.array_equal(got, _sa(ctx, A, "sjlt", m, seed=5, t=3, s=s))


@pytest.mark.parametrize("n,d,m", [(100, 3, 16), (3000, 64, 256), (5001, 129, 200)])
def test_gaussian_sketch(ctx, n, d, m):
    from oracle import draws, sketch
    say("gauss sketch", n, d, m)
    A = np.random.default_rng(n).standard_normal((n, d))
    got = _sa(ctx, A, "gaussian", m, seed=21, t=2)
    ref = sketch.gaussian_sketch(A, m, 21, 2)
    G = draws.gaussian_matrix(21, 2, m, n)
    # FP64 normals within a few ulp of the oracle's, FP64 products and sums in any order
    bound = (4 * n + 16) * EPS * (np.abs(G) @ np.abs(A))
    assert np.all(np.abs(got - ref) <= bound)


# ----------------------------------------------------------------------------------------------
# factor
# ----------------------------------------------------------------------------------------------
def factor_amplification(Ro, kappa, mode):
    """How the factor's forward error grows with kappa: kappa for a backward-stable R (Householder,
    CholeskyQR2, shifted CholeskyQR3: lsq_factor's default), kappa^2 for the one-pass Cholesky factor of
    X^T X (option 5)."""
    one_pass = mode == 5
    return kappa * kappa if one_pass else kappa


@pytest.mark.parametrize("mode", [0, 5])
@pytest.mark.parametrize("m,d,kappa", [(16, 3, 10.0), (256, 64, 1e3), (700, 129, 1e6), (1500, 300, 1e4),
                                       (2048, 512, 1e8), (4100, 1024, 1e4)])
def test_factor(ctx, m, d, kappa, mode):
    from oracle.householder import householder_qr
    from synth import make_problem
    torch = _torch()
    say("factor", m, d, kappa, mode)
    X = make_problem(m, d, kappa, seed=m)["A"]
    R = torch.empty((d, d), dtype=torch.float64, device="cuda")
    W = torch.empty((d, d), dtype=torch.float64, device="cuda")
    ctx.set_option("factor", mode)
    try:
        ctx.factor(dev(X), R, W)
    finally:
        ctx.set_option("factor", 0)
    Rg, Wg = host(R), host(W)
    Ro = householder_qr(X)
    amp = factor_amplification(Ro, kappa, mode)
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    # R^T R reproduces X^T X to O(eps) relative to ||X||^2 (the Gram rounding and the Cholesky's backward
    # error; QR's backward error for the two-pass forms)
    nx2 = np.linalg.norm(X, 2) ** 2
    assert np.abs(Rg.T @ Rg - X.T @ X).max() <= 50 * m * EPS * nx2
    # R itself is unique; rows agree to O(eps kappa) (O(eps kappa^2) for the Cholesky factor of X^T X)
    assert np.abs(Rg - Ro).max() <= 50 * m * EPS * amp * np.abs(Ro).max()
    # X R^{-1} has orthonormal columns to the same order
    Q = X @ Wg
    assert np.abs(Q.T @ Q - np.eye(d)).max() <= 1e3 * m * EPS * amp


def test_factor_rank_deficient(ctx):
    from paper_1911_02675_amd import lsq
    torch = _torch()
    X = np.random.default_rng(0).standard_normal((200, 10))
    X[:, 7] = X[:, 2]
    R = torch.empty((10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(lsq.LsqError) as e:
        ctx.factor(dev(X), R, None)
    assert e.value.status == lsq.LSQ_ERR_RANK


# ----------------------------------------------------------------------------------------------
# solves
# ----------------------------------------------------------------------------------------------
def _floor(A, y):
    """Disagreement of two backward-stable FP64 solvers (Householder, LAPACK SVD) in e_A."""
    from oracle.solve import a_norm_error, lstsq_householder
    x1 = lstsq_householder(A, y, block_rows=8192)
    x2 = np.linalg.lstsq(A, y, rcond=None)[0]
    return x1, a_norm_error(A, x2, x1)


@pytest.mark.parametrize("kind,s", [("srht", 1), ("sjlt", 4), ("gaussian", 1)])
def test_pcg_small_config(ctx, kind, s):
    """n = 4096, d = 64, kappa = 1e3, m = 4d, noise 0.01: PCG to relative A-norm error 1e-10."""
    from oracle.pcg import pcg, sketch_factor
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    torch = _torch()
    say("pcg small", kind)
    P = make_problem(4096, 64, 1e3, sigma=0.01, seed=1)
    A, y = P["A"], P["y"]
    xs, fl = _floor(A, y)
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    desc = lsq.sketch_desc(kind, 256, seed=3, s=s)
    st, info = ctx.pcg_solve(dev(A), dev(y), desc, x, tol=1e-10)
    e = a_norm_error(A, host(x), xs)
    say("  e_A", e, "floor", fl, "iters", info.iters)
    assert e <= max(1e-10, 4 * fl)
    # same sketch on the oracle: iteration counts agree to within a couple of steps
    _, its = pcg(A, y, sketch_factor(A, kind, 256, 3, s=s), tol=1e-10)
    assert abs((len(its) - 1) - info.iters) <= 2


@pytest.mark.parametrize("n,d,m,kind,kappa", [(30001, 128, 512, "srht", 1e4), (20000, 100, 400, "sjlt", 1e6),
                                              (16384, 256, 1024, "srht", 1e2), (9000, 33, 140, "gaussian", 1e5)])
def test_pcg_medium(ctx, n, d, m, kind, kappa):
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    torch = _torch()
    say("pcg medium", n, d, m, kind, kappa)
    P = make_problem(n, d, kappa, sigma=0.01, seed=n)
    A, y = P["A"], P["y"]
    xs, fl = _floor(A, y)
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    st, info = ctx.pcg_solve(dev(A), dev(y), lsq.sketch_desc(kind, m, seed=9, s=2), x, tol=1e-10)
    e = a_norm_error(A, host(x), xs)
    say("  e_A", e, "floor", fl, "iters", info.iters)
    assert e <= max(1e-10, 4 * fl)


@pytest.mark.parametrize("inner_f32,kappa", [(0, 1e4), (0, 1e6), (1, 1e3)])
def test_pcg_mixed_fp32_storage(ctx, inner_f32, kappa):
    """Precision form: FP32 A (the problem is A32 promoted exactly), FP32 SRHT, FP64 residual + IR."""
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_planted
    torch = _torch()
    say("mixed", inner_f32, kappa)
    P = make_planted(1 << 15, 128, kappa, sigma=0.01, seed=4, want64=False, want32=True)
    A32, y, xs = P["A32"], P["y32"], P["x_star"]
    x = torch.zeros(128, dtype=torch.float64, device="cuda")
    desc = lsq.sketch_desc("srht", 512, seed=2, compute="f32")
    st, info = ctx.pcg_solve(dev(A32), dev(y), desc, x, tol=1e-10, mixed=1, inner_f32=inner_f32,
                             max_refine=30)
    A64 = A32.astype(np.float64)
    e = a_norm_error(A64, host(x), xs)
    say("  e_A", e, "iters", info.iters, "refinements", info.refinements)
    floor = 4 * EPS * kappa * np.linalg.norm(y - A64 @ xs) / np.linalg.norm(A64 @ xs)
    assert e <= max(1e-10, floor)


@pytest.mark.parametrize("mixed,compute", [(0, "f64"), (1, "f32"), (1, "f64")])
def test_pcg_first_gradient_from_pass_a(ctx, mixed, compute):
    """From x_0 = 0 with the SRHT in its vector form, the first gradient A^T y comes from the sketch's
    first pass.  A start of 1e-200 e_0 has the same first residual to rounding but takes it from a pass
    of its own (plain, or double-double in the mixed form), with the same sketch: the iterates after three
    fixed iterations agree to rounding.  With lda not a multiple of 16 bytes the sketch takes its general
    form and the solve a plain first pass; it converges to the same solution.  The mixed form runs with
    an FP32 and with an FP64 transform of its FP32 A (the latter converts the loaded rows to FP64)."""
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    torch = _torch()
    n, d, m = 30001, 128, 512
    say("first gradient", mixed, compute)
    P = make_problem(n, d, 1e4, sigma=0.01, seed=77)
    A, y = P["A"], P["y"]
    if mixed:
        A = A.astype(np.float32).astype(np.float64)
    dt = torch.float32 if mixed else torch.float64
    Ad = torch.tensor(A, dtype=dt, device="cuda")
    yd = dev(y)
    desc = lsq.sketch_desc("srht", m, seed=5, compute=compute)
    xs = []
    for x0 in (0.0, 1e-200):
        x = torch.zeros(d, dtype=torch.float64, device="cuda")
        x[0] = x0
        ctx.pcg_solve(Ad, yd, desc, x, tol=1e-10, max_iter=3, stop_rule=1, mixed=mixed, max_refine=1)
        xs.append(host(x))
    assert np.linalg.norm(xs[0] - xs[1]) <= 1e-11 * np.linalg.norm(xs[1])
    wide = torch.zeros((n, d + 1), dtype=dt, device="cuda")
    wide[:, :d] = Ad
    xf, fl = _floor(A, y)
    for Am in (Ad, wide[:, :d]):  # lda = d, d + 1
        x = torch.zeros(d, dtype=torch.float64, device="cuda")
        ctx.pcg_solve(Am, yd, desc, x, tol=1e-10, mixed=mixed, max_refine=30)
        assert a_norm_error(A, host(x), xf) <= max(1e-10, 4 * fl)


def test_pcg_planted_exact(ctx):
    """Planted problem (noise orthogonal to range(A)): x* is known exactly."""
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_planted
    torch = _torch()
    P = make_planted(1 << 16, 200, 1e5, sigma=0.01, seed=8)
    A, y, xs = P["A64"], P["y64"], P["x_star"]
    x = torch.zeros(200, dtype=torch.float64, device="cuda")
    trace = torch.zeros(201, dtype=torch.float64, device="cuda")
    st, info = ctx.pcg_solve(dev(A), dev(y), lsq.sketch_desc("srht", 800, seed=1), x, tol=1e-10,
                             x_ref=dev(xs), err_trace=trace)
    e = a_norm_error(A, host(x), xs)
    say("planted e_A", e, info.iters)
    assert e <= 1e-10
    tr = host(trace)[: info.iters + 1]
    assert abs(tr[0] - 1.0) < 1e-12 and tr[-1] <= 1e-10 * 1.5


def test_pcg_errors(ctx):
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    torch = _torch()
    P = make_problem(2000, 20, 1e8, seed=3)
    A, y = dev(P["A"]), dev(P["y"])
    x = torch.zeros(20, dtype=torch.float64, device="cuda")
    for desc, code in [(lsq.sketch_desc("srht", 10), lsq.LSQ_ERR_INVALID_ARG),
                       (lsq.sketch_desc("srht", 4096), lsq.LSQ_ERR_INVALID_ARG),
                       (lsq.sketch_desc("sjlt", 64, s=0), lsq.LSQ_ERR_INVALID_ARG),
                       (lsq.sketch_desc("sjlt", 64, s=65), lsq.LSQ_ERR_INVALID_ARG)]:
        st, _ = ctx.pcg_solve(A, y, desc, x, raise_on_error=False)
        assert st == code
    assert np.all(host(x) == 0)  # argument errors leave x untouched
    st, info = ctx.pcg_solve(A, y, lsq.sketch_desc("srht", 80), x, tol=1e-10, max_iter=3,
                             raise_on_error=False)
    assert st == lsq.LSQ_ERR_NOT_CONVERGED and info.iters == 3
    Xb = P["A"].copy()
    Xb[:, 5] = Xb[:, 9]
    st, _ = ctx.pcg_solve(dev(Xb), y, lsq.sketch_desc("gaussian", 80), x, raise_on_error=False)
    assert st == lsq.LSQ_ERR_RANK


@pytest.mark.parametrize("kind,s", [("srht", 1), ("sjlt", 2), ("gaussian", 1)])
def test_pcg_nonfinite(ctx, kind, s):
    """A NaN or an infinity in A reaches S A (every embedding mixes each row of A into some row of S A)
    and is reported as such before the factorization; one in y reaches the first residual."""
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    torch = _torch()
    say("nonfinite", kind)
    P = make_problem(3000, 20, 1e3, seed=5)
    for where, val, a32 in [("A", np.nan, False), ("A", np.inf, False), ("y", np.nan, False), ("y", -np.inf, False),
                            ("A", np.nan, True), ("y", np.inf, True)]:
        A, y = P["A"].copy(), P["y"].copy()
        if where == "A":
            A[1234, 7] = val
        else:
            y[777] = val
        Ad = dev(A.astype(np.float32)) if a32 else dev(A)
        x = torch.zeros(20, dtype=torch.float64, device="cuda")
        st, _ = ctx.pcg_solve(Ad, dev(y), lsq.sketch_desc(kind, 80, seed=2, s=s,
                                                          compute="f32" if a32 and kind == "srht" else "f64"),
                              x, mixed=int(a32), raise_on_error=False)
        assert st == lsq.LSQ_ERR_NONFINITE, (where, val, a32, st)
    SA = np.random.default_rng(1).standard_normal((100, 20))
    SA[3, 4] = np.nan
    R = torch.empty((20, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(lsq.LsqError) as e:
        ctx.factor(dev(SA), R, None)
    assert e.value.status == lsq.LSQ_ERR_NONFINITE


def test_pcg_plain_verified_beyond_fp64_floor(ctx):
    """Plain FP64 form at kappa = 1e8 on a planted noisy problem (x* exact): PCG's recursively updated
    residual keeps meeting the proxy after the true error has stalled near the FP64 floor, so the result
    is measured with a double-double residual.  With one correction solve the status must not claim the
    tolerance unless x meets it; with the default budget, residual replacement reaches it."""
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_planted
    torch = _torch()
    n, d, m = 1 << 16, 128, 1024
    P = make_planted(n, d, 1e8, sigma=0.01, seed=93)
    A, y, xs = P["A64"], P["y64"], P["x_star"]
    Ad, yd = dev(A), dev(y)
    for max_refine in (1, 8):
        x = torch.zeros(d, dtype=torch.float64, device="cuda")
        st, info = ctx.pcg_solve(Ad, yd, lsq.sketch_desc("srht", m, seed=4), x, tol=1e-10, max_iter=300,
                                 max_refine=max_refine, raise_on_error=False)
        e = a_norm_error(A, host(x), xs)
        say("  plain kappa 1e8, max_refine", max_refine, "status", st, "solves", info.refinements,
            "iters", info.iters, "estimate", info.est_rel_err, "e_A", e)
        assert st in (lsq.LSQ_OK, lsq.LSQ_ERR_NOT_CONVERGED)
        if st == lsq.LSQ_OK:
            assert e <= 1e-10
    assert st == lsq.LSQ_OK and e <= 1e-10


# ----------------------------------------------------------------------------------------------
# IHS / Polyak-IHS
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("kind,beta,refresh", [("gaussian", 0.0, 1), ("gaussian", 0.5, 1), ("srht", 0.1, 1),
                                               ("srht", 0.0, 0)])
def test_ihs_iterates(ctx, kind, beta, refresh):
    """Same draws on both sides: the iterates agree to the rounding of the sketches."""
    from oracle import theory
    from oracle.ihs import ihs
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    torch = _torch()
    say("ihs", kind, beta, refresh)
    n, d, m, T = 4096, 32, 128, 8
    P = make_problem(n, d, 1e4, sigma=0.01, seed=6)
    A, y = P["A"], P["y"]
    if kind == "gaussian":
        t1, t2 = theory.theta_gaussian(m, d)
        mu = t1 / t2
    else:
        t1, t2 = theory.srht_thetas_scaled(n, d, m)
        mu = t1 / t2
    its = ihs(A, y, kind, m, seed=77, mu=mu, beta=beta, iters=T, refresh=bool(refresh))
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    info = ctx.ihs_solve(dev(A), dev(y), lsq.sketch_desc(kind, m, seed=77), x, iters=T, beta=beta,
                         refresh=refresh, mu_rule=0)
    assert abs(info.mu - mu) <= 1e-12 * mu
    xo = its[-1]
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    diff = a_norm_error(A, host(x), xo) * np.linalg.norm(A @ xo) / np.linalg.norm(A @ xs)
    say("  diff", diff, "err", a_norm_error(A, xo, xs))
    # every sketch is FP64 on both sides (the Gaussian normals within a few ulp): iterates agree to the
    # rounding of the factorizations and passes
    tol = 1e-10
    assert diff <= tol
