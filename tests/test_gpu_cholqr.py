"""GPU parity of the Gram-matrix factorization (CholeskyQR2, and shifted CholeskyQR3 above the
Householder limit) against the oracle's Householder QR, through lsq_factor, plus the solver on a
sketch larger than the Householder limit.  Bounds as for the Householder factor: R^T R reproduces
X^T X to 50 m eps ||X||^2, R matches the oracle's R to 50 m eps kappa max|R|, X R^{-1} is orthonormal
to 1e3 m eps kappa."""
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


def _check(X, Rg, Wg, kappa):
    from oracle.householder import householder_qr
    m, d = X.shape
    Ro = householder_qr(X)
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    nx2 = np.linalg.norm(X, 2) ** 2
    assert np.abs(Rg.T @ Rg - X.T @ X).max() <= 50 * m * EPS * nx2
    assert np.abs(Rg - Ro).max() <= 50 * m * EPS * kappa * np.abs(Ro).max()
    Q = X @ Wg
    assert np.abs(Q.T @ Q - np.eye(d)).max() <= 1e3 * m * EPS * kappa


@pytest.mark.parametrize("m,d,kappa,mode", [(300, 64, 1e3, 0), (700, 129, 1e6, 0), (1500, 300, 1e4, 0),
                                            (1500, 300, 1e4, 1), (9000, 200, 1e4, 0), (12000, 96, 1e9, 0),
                                            (4100, 1024, 1e5, 0)])
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
        _check(X, R.cpu().numpy(), W.cpu().numpy(), kappa)
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
            ctx.set_option("factor", 4)  # 0..3 are the factor forms
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
