"""Haar embedding on the GPU (S = Q^T of the positive-diagonal QR of the Gaussian draws, formed as
R^{-T} (g A)) against the oracle (numpy QR of the same counter-based draws).

The device's normals are FP64 values within a few ulp of the oracle's, so S differs from the oracle's by
the rounding of the two factorizations (Cholesky of g g^T on the device, Householder QR of g^T in the
oracle), about m u kappa(g)^2 with kappa(g) <= 3 here; the orthonormality of the rows is checked on the
device result directly (A = I gives S A = S), independently of the draws."""
import math
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sa(ctx, A, m, seed, t=0):
    import torch
    from paper_1911_02675_amd import lsq
    n, d = A.shape
    SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
    ctx.sketch(dev(A), dev(np.zeros(n)), lsq.sketch_desc("haar", m, seed=seed, t=t), SA)
    torch.cuda.synchronize()
    return SA.cpu().numpy()


@pytest.mark.parametrize("n,m", [(500, 100), (333, 65), (1024, 256)])
def test_haar_rows_orthonormal(ctx, n, m):
    say("haar orthonormal", n, m)
    S = _sa(ctx, np.eye(n), m, seed=3, t=1)
    err = np.max(np.abs(S @ S.T - np.eye(m)))
    say("  max |S S^T - I|", err)
    assert err <= 64 * m * EPS


@pytest.mark.parametrize("n,d,m", [(3000, 20, 100), (5001, 7, 65), (20001, 64, 700), (1 << 14, 130, 1024)])
def test_haar_sketch_parity(ctx, n, d, m):
    from oracle import sketch
    say("haar sketch", n, d, m)
    A = np.random.default_rng(n + d).standard_normal((n, d))
    got = _sa(ctx, A, m, seed=21, t=2)
    ref = sketch.haar_sketch(A, m, 21, 2)
    # S ~ g / sqrt(n): the FP64 rounding of the products and of the factorizations, m u kappa(g)^2 per
    # entry of S, summed over the column of A
    bound = 64 * m * EPS * (np.abs(A).sum(axis=0)[None, :] / math.sqrt(n) + np.linalg.norm(A, axis=0)[None, :])
    r = np.max(np.abs(got - ref) / bound)
    say("  max err / bound", r)
    assert r <= 1.0


def test_haar_limits(ctx):
    import torch
    from paper_1911_02675_amd import lsq
    A = dev(np.ones((100, 4)))
    SA = torch.empty((200, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(lsq.LsqError) as e:
        ctx.sketch(A, dev(np.zeros(100)), lsq.sketch_desc("haar", 200, seed=1), SA)  # m > n
    assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    with pytest.raises(lsq.LsqError) as e:
        ctx.sketch(A, dev(np.zeros(100)), lsq.sketch_desc("haar", 20, seed=1, compute="f32"), SA)
    assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    with pytest.raises(lsq.LsqError) as e:
        ctx.sketch(A, dev(np.zeros(100)), lsq.sketch_desc("haar", 26, seed=1), SA)  # m > n/4
    assert e.value.status == lsq.LSQ_ERR_UNSUPPORTED


def test_haar_pcg_and_refreshed_ihs(ctx):
    import torch
    from oracle import theory
    from oracle.ihs import ihs
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    n, d, m, T = 4096, 32, 128, 8
    P = make_problem(n, d, 1e4, sigma=0.01, seed=7)
    A, y = P["A"], P["y"]
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    # PCG with a Haar preconditioner reaches the tolerance
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    st, info = ctx.pcg_solve(dev(A), dev(y), lsq.sketch_desc("haar", m, seed=5), x, tol=1e-10, max_iter=100)
    e = a_norm_error(A, x.cpu().numpy(), xs)
    say("  haar pcg: iters", info.iters, "e_A", e)
    assert st == lsq.LSQ_OK and e <= 1e-10
    # refreshed IHS with the Section 2 Haar step against the oracle's iterates
    t1, t2 = theory.theta_haar(n, d, m)
    mu = t1 / t2
    its = ihs(A, y, "haar", m, seed=77, mu=mu, iters=T, refresh=True)
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    info = ctx.ihs_solve(dev(A), dev(y), lsq.sketch_desc("haar", m, seed=77), x, iters=T, refresh=1, mu_rule=0)
    assert abs(info.mu - mu) <= 1e-12 * mu
    xo = its[-1]
    diff = a_norm_error(A, x.cpu().numpy(), xo) * np.linalg.norm(A @ xo) / np.linalg.norm(A @ xs)
    say("  haar ihs: diff", diff, "err", a_norm_error(A, xo, xs))
    assert diff <= 1e-10
