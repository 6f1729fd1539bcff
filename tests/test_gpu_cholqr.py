"""GPU parity of the Gram-matrix factorization (the one-pass Cholesky factor of X^T X, CholeskyQR2, and
shifted CholeskyQR3 above the Householder limit) against the oracle's Householder QR, through lsq_factor,
plus the solver on a sketch larger than the Householder limit.  Bounds: R^T R reproduces X^T X to
50 m eps ||X||^2; R matches the oracle's R to 50 m eps a max|R| and X R^{-1} is orthonormal to
1e3 m eps a, with a = kappa for the backward-stable forms and kappa^2 for the one-pass factor."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_02675_amd import lsq
    c = lsq.Context()
    yield c
    c.close()


def factor_amplification(Ro, kappa, mode):
    """kappa for a backward-stable R (lsq_factor's default); kappa^2 for the one-pass Cholesky factor of
    X^T X (option 5)."""
    one_pass = mode == 5
    return kappa * kappa if one_pass else kappa


def _check(X, Rg, Wg, kappa, mode):
    from oracle.householder import householder_qr
    m, d = X.shape
    Ro = householder_qr(X)
    amp = factor_amplification(Ro, kappa, mode)
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    nx2 = np.linalg.norm(X, 2) ** 2
    assert np.abs(Rg.T @ Rg - X.T @ X).max() <= 50 * m * EPS * nx2
    assert np.abs(Rg - Ro).max() <= 50 * m * EPS * amp * np.abs(Ro).max()
    Q = X @ Wg
    assert np.abs(Q.T @ Q - np.eye(d)).max() <= 1e3 * m * EPS * amp


# lsq_factor: 0 CholeskyQR2 with fallbacks, 1 Householder, 4 CholeskyQR2 forced, 5 one pass forced
@pytest.mark.parametrize("m,d,kappa,mode", [(300, 64, 1e3, 0), (700, 129, 1e6, 0), (700, 129, 1e6, 4),
                                            (1500, 300, 1e4, 0), (1500, 300, 1e4, 1), (1500, 300, 1e4, 4),
                                            (1500, 300, 1e4, 5), (9000, 200, 1e4, 0), (9000, 200, 1e4, 4),
                                            (12000, 96, 1e9, 0), (4100, 1024, 1e5, 0), (4100, 1024, 1e5, 4),
                                            (20000, 256, 1e7, 0)])
def test_factor_paths(ctx, m, d, kappa, mode):
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_problem
    say("factor path", m, d, kappa, mode)
    ctx.set_option("factor", mode)
    try:
        X = make_problem(m, d, kappa, seed=m + d)["A"]
        R = torch.empty((d, d), dtype=torch.float64, device="cuda")
        W = torch.empty((d, d), dtype=torch.float64, device="cuda")
        ctx.factor(torch.from_numpy(X).cuda(), R, W)
        torch.cuda.synchronize()
        _check(X, R.cpu().numpy(), W.cpu().numpy(), kappa, mode)
    finally:
        ctx.set_option("factor", 0)


def test_factor_limits_and_rank(ctx):
    import torch

    from paper_1911_02675_amd import lsq
    rng = np.random.default_rng(4)
    X = rng.standard_normal((9000, 12))
    X[:, 5] = X[:, 1]
    R = torch.empty((12, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(lsq.LsqError) as e:
        ctx.factor(torch.from_numpy(X).cuda(), R, None)  # rank deficient above the Householder limit
    assert e.value.status == lsq.LSQ_ERR_RANK
    ctx.set_option("factor", 1)
    try:
        X = rng.standard_normal((9000, 12))
        with pytest.raises(lsq.LsqError) as e:
            ctx.factor(torch.from_numpy(X).cuda(), R, None)
        assert e.value.status == lsq.LSQ_ERR_UNSUPPORTED
    finally:
        ctx.set_option("factor", 0)
    try:
        with pytest.raises(lsq.LsqError) as e:
            ctx.set_option("factor", 6)  # 0..5 are the factor forms
        assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    finally:
        ctx.set_option("factor", 0)


def test_pcg_with_sketch_above_householder_limit(ctx):
    import torch

    from oracle.solve import a_norm_error, lstsq_householder
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    n, d, m = 1 << 16, 512, 10240
    P = make_problem(n, d, 1e5, sigma=0.01, seed=77)
    A, y = P["A"], P["y"]
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    st, info = ctx.pcg_solve(torch.from_numpy(A).cuda(), torch.from_numpy(y).cuda(),
                             lsq.sketch_desc("srht", m, seed=3), x, tol=1e-10)
    torch.cuda.synchronize()
    xs = lstsq_householder(A, y, block_rows=8192)
    e = a_norm_error(A, x.cpu().numpy(), xs)
    say("  PCG m = 10240: iterations", info.iters, "e_A", e)
    assert e <= 1e-10
    assert info.iters <= 20  # rho = d/m = 0.05: about 8 iterations by the bound


@pytest.mark.parametrize("kappa", [1e4, 1e7])
def test_pcg_one_pass_factor_iterations(ctx, kappa):
    """PCG takes the one-pass Cholesky factor of H_S when the first factor's diagonal spread is at most
    2e5 (kappa = 1e4 here) and CholeskyQR2 above (kappa = 1e7: spread about 4e5): the iteration count and
    the accuracy equal those with CholeskyQR2 forced (option 4), and the one-pass factor (option 5) alone
    gives the same count at kappa = 1e7 too."""
    import torch

    from oracle.solve import a_norm_error, lstsq_householder
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    n, d, m = 1 << 16, 256, 6144
    P = make_problem(n, d, kappa, sigma=0.01, seed=78)
    A, y = P["A"], P["y"]
    xs = lstsq_householder(A, y, block_rows=8192)
    Ag, yg = torch.from_numpy(A).cuda(), torch.from_numpy(y).cuda()
    res = {}
    try:
        for mode in (0, 4, 5):
            ctx.set_option("factor", mode)
            x = torch.zeros(d, dtype=torch.float64, device="cuda")
            st, info = ctx.pcg_solve(Ag, yg, lsq.sketch_desc("srht", m, seed=5), x, tol=1e-10)
            torch.cuda.synchronize()
            e = a_norm_error(A, x.cpu().numpy(), xs)
            say("  kappa", kappa, "factor option", mode, "iterations", info.iters, "e_A", e)
            assert st == lsq.LSQ_OK and e <= 1e-10
            res[mode] = info.iters
    finally:
        ctx.set_option("factor", 0)
    assert abs(res[0] - res[4]) <= 1 and abs(res[5] - res[4]) <= 1
