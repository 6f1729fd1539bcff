"""Pins of the oracle's SVD (LSRN) preconditioner and minimum-norm solution.

  full rank      min_norm_lstsq equals the Householder solve; P P^T equals R^{-1} R^{-T}
  duplicate col  for A = [B, b_0] (b_0 = first column of B repeated) the minimum-norm solution splits the
                 first coefficient of B's solution equally between the two copies (closed form)
  Penrose        with a rank-deficient S A, P P^T is the pseudo-inverse of H_S: H P P^T H = H and
                 P P^T H P P^T = P P^T
  PCG            with P, PCG from x_0 = 0 reaches the minimum-norm solution of a rank-deficient problem
"""
import numpy as np

from oracle.householder import householder_qr
from oracle.pcg import pcg, pcg_svd, svd_preconditioner
from oracle.solve import lstsq_householder, min_norm_lstsq
from synth import make_problem


def test_min_norm_full_rank_and_duplicate_column():
    P = make_problem(600, 12, 1e4, seed=41)
    A, y = P["A"], P["y"]
    xh = lstsq_householder(A, y)
    assert np.linalg.norm(min_norm_lstsq(A, y) - xh) <= 1e-9 * np.linalg.norm(xh)
    Ad = np.hstack([A, A[:, :1]])
    x = min_norm_lstsq(Ad, y)
    expect = np.concatenate([[xh[0] / 2], xh[1:], [xh[0] / 2]])
    assert np.linalg.norm(x - expect) <= 1e-9 * np.linalg.norm(expect)


def test_svd_preconditioner_full_rank_and_penrose():
    rng = np.random.default_rng(2)
    SA = make_problem(200, 10, 1e5, seed=42)["A"]
    R = householder_qr(SA)
    Pm = svd_preconditioner(SA)
    M = np.linalg.solve(R, np.linalg.solve(R, np.eye(10)).T)  # R^{-1} R^{-T}
    assert np.linalg.norm(Pm @ Pm.T - M) <= 1e-8 * np.linalg.norm(M)
    # Penrose conditions hold to about u kappa(S A)^2: a moderately conditioned block keeps them tight
    SA = make_problem(200, 10, 1e2, seed=44)["A"]
    SAd = np.hstack([SA, SA[:, 3:4], SA[:, :2] @ rng.standard_normal((2, 1))])
    H = SAd.T @ SAd
    Pd = svd_preconditioner(SAd)
    assert Pd.shape[1] == 10  # rank
    G = Pd @ Pd.T
    assert np.linalg.norm(H @ G @ H - H) <= 1e-9 * np.linalg.norm(H)
    assert np.linalg.norm(G @ H @ G - G) <= 1e-9 * np.linalg.norm(G)


def test_pcg_svd_reaches_min_norm_solution():
    rng = np.random.default_rng(4)
    P = make_problem(3000, 20, 1e3, seed=43)
    A = np.hstack([P["A"], P["A"][:, 5:6], P["A"][:, :3] @ rng.standard_normal((3, 1))])
    y = P["y"]
    S = rng.standard_normal((200, 3000)) / np.sqrt(200)
    Pm = svd_preconditioner(S @ A)
    x, its = pcg_svd(A, y, Pm, tol=1e-12, max_iter=100)
    xm = min_norm_lstsq(A, y)
    assert np.linalg.norm(x - xm) <= 1e-8 * np.linalg.norm(xm)
    # full rank: the same iterates as the triangular preconditioner (same H_S^{-1})
    R = householder_qr(S @ P["A"])
    Pf = svd_preconditioner(S @ P["A"])
    _, it1 = pcg(P["A"], y, R, fixed_iters=6)
    _, it2 = pcg_svd(P["A"], y, Pf, fixed_iters=6)
    for a, b in zip(it1, it2):
        assert np.linalg.norm(a - b) <= 1e-8 * max(np.linalg.norm(it1[-1]), 1.0)


def test_qrcp_preconditioner():
    """Column-pivoted QR (scipy): |R_kk| non-increasing, S A P = Q R; W W^T = H_S^{-1} at full rank; with
    dependent columns the rank is found and PCG gives the basic solution: zero on the dropped columns and
    the least-squares residual (normal equations on every column)."""
    import scipy.linalg

    from oracle.pcg import pcg_with, qrcp_preconditioner
    rng = np.random.default_rng(6)
    SA = make_problem(300, 12, 1e3, seed=45)["A"]
    Q, R, piv = scipy.linalg.qr(SA, mode="economic", pivoting=True)
    dg = np.abs(np.diag(R))
    assert np.all(dg[1:] <= dg[:-1] * (1 + 1e-12))
    assert np.linalg.norm(SA[:, piv] - Q @ R) <= 1e-13 * np.linalg.norm(SA)
    W, r, _ = qrcp_preconditioner(SA)
    M = np.linalg.inv(SA.T @ SA)
    assert r == 12 and np.linalg.norm(W @ W.T - M) <= 1e-9 * np.linalg.norm(M)
    P = make_problem(2000, 16, 1e2, seed=46)
    A = np.hstack([P["A"], P["A"][:, 2:3], P["A"][:, :2] @ rng.standard_normal((2, 1))])
    y = P["y"]
    S = rng.standard_normal((150, 2000)) / np.sqrt(150)
    W, r, piv = qrcp_preconditioner(S @ A)
    assert r == 16
    x, _ = pcg_with(A, y, lambda v: W @ (W.T @ v), tol=1e-13, max_iter=100)
    assert np.all(x[piv[r:]] == 0.0)
    assert np.linalg.norm(A.T @ (A @ x - y)) <= 1e-9 * np.linalg.norm(A.T @ y)
    xm = min_norm_lstsq(A, y)
    assert abs(np.linalg.norm(A @ x - y) - np.linalg.norm(A @ xm - y)) <= 1e-10 * np.linalg.norm(y)
