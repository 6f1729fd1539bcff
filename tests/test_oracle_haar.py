"""Pins of the oracle's Haar embedding (Section 2: orthonormal rows, uniformly distributed span).

  definition     S S^T = I_m; S G is upper triangular with a positive diagonal (S = Q^T of the
                 positive-diagonal QR of the Gaussian draws G), so S spans exactly the draws' columns
  uniformity     E[S^T S] = (m/n) I_n, and ||S e_1||^2 ~ Beta(m/2, (n-m)/2): mean m/n, variance
                 2 m (n - m) / (n^2 (n + 2)), over independent refresh counters t
  inverse moment E[C_S^{-1}] = (n - d - 1)/(m - d - 1) I exactly (matrix-variate beta), whose large-size
                 limit is Section 2's theta_1 ~ (n - d)/(m - d)
"""
import numpy as np

from oracle import draws, sketch, theory


def test_haar_rows_orthonormal_and_span_the_draws():
    n, m = 300, 40
    S = sketch.haar_matrix(n, m, seed=5, t=2)
    assert S.shape == (m, n)
    assert np.max(np.abs(S @ S.T - np.eye(m))) <= 1e-13
    G = draws.gaussian_normals(5, 2, np.arange(m)[None, :], np.arange(n)[:, None])
    T = S @ G  # = R of the QR of G
    assert np.max(np.abs(np.tril(T, -1))) <= 1e-12 * np.max(np.abs(T))
    assert np.all(np.diag(T) > 0)
    # S A equals the dense product
    A = np.random.default_rng(0).standard_normal((n, 7))
    assert np.allclose(sketch.sketch(A, "haar", m, 5, 2), S @ A, rtol=0, atol=1e-13)


def test_haar_is_uniform():
    n, m, N = 12, 4, 6000
    acc = np.zeros((n, n))
    v = np.empty(N)
    for t in range(N):
        S = sketch.haar_matrix(n, m, seed=9, t=t)
        P = S.T @ S
        acc += P
        v[t] = P[0, 0]
    mean = acc / N
    # each diagonal entry of P is Beta(m/2, (n-m)/2) distributed (sd ~ 0.12 here)
    var = 2 * m * (n - m) / (n * n * (n + 2))
    se = np.sqrt(var / N)
    assert np.max(np.abs(np.diag(mean) - m / n)) <= 5 * se
    assert np.max(np.abs(mean - np.diag(np.diag(mean)))) <= 5 * se
    assert abs(v.mean() - m / n) <= 5 * se
    assert abs(v.var() / var - 1.0) <= 0.1


def test_haar_inverse_moment_exact():
    n, d, m, N = 20, 3, 10, 6000
    U, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n, d)))
    tr = np.empty(N)
    for t in range(N):
        S = sketch.haar_matrix(n, m, seed=11, t=t)
        tr[t] = np.trace(np.linalg.inv(U.T @ S.T @ S @ U)) / d
    exact = theory.theta1_haar_exact(n, d, m)
    assert abs(tr.mean() - exact) <= 4 * tr.std() / np.sqrt(N)
    # the paper's approximation is the large-size limit of the exact value
    t1, _ = theory.theta_haar(20000, 5, 400)
    assert abs(theory.theta1_haar_exact(20000, 5, 400) / t1 - 1.0) <= 3e-3
