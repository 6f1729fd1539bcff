"""Pins of the oracle's Haar embedding (Section 2: orthonormal rows, uniformly distributed span).

  definition     S S^T = I_m; S G is upper triangular with a positive diagonal (S = Q^T of the
                 positive-diagonal QR of the Gaussian draws G), so S spans exactly the draws' columns
  uniformity     E[S^T S] = (m/n) I_n, and ||S e_1||^2 ~ Beta(m/2, (n-m)/2): mean m/n, variance
                 2 m (n - m) / (n^2 (n + 2)), over independent refresh counters t
  inverse moment E[C_S^{-1}] = (n - d - 1)/(m - d - 1) I exactly (matrix-variate beta), whose large-size
                 limit is Section 2's theta_1 ~ (n - d)/(m - d)
  second moment  d^{-1} tr E[C_S^{-2}] equals the closed form derived from the Wishart moments
                 (theory.theta2_haar_exact), checked by Monte Carlo over explicit Haar matrices; Section 2's
                 theta_2 ~ (n - d)(d^2 + m n - 2 d m)/(m - d)^3 is its large-size limit, checked at a size
                 where every term of the approximation moves it by 20 % or more
  SRHT moments   with S = m^{-1/2} R H E (S S^T = (N/m) I), d^{-1} tr E[C_S^{-1}] and d^{-1} tr E[C_S^{-2}]
                 over explicit SRHT matrices equal (m/N) and (m/N)^2 times the Haar values for
                 orthonormal rows (Section 2: the SRHT obeys the Haar trace formulas), and
                 theory.srht_thetas_scaled is that rescaling of Section 2's approximations
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


def _inverse_moments(U, mats):
    """d^{-1} tr C_S^{-1} and d^{-1} tr C_S^{-2} for each explicit S (Condition 2.1's trace form)."""
    d = U.shape[1]
    t1, t2 = [], []
    for S in mats:
        Ci = np.linalg.inv(U.T @ S.T @ S @ U)
        t1.append(np.trace(Ci) / d)
        t2.append(np.trace(Ci @ Ci) / d)
    return np.array(t1), np.array(t2)


def test_haar_second_inverse_moment_exact():
    # m - d - 3 = 14 leaves the variance of tr C_S^{-2} finite, so the standard error is meaningful
    n, d, m, N = 40, 3, 20, 4000
    U, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n, d)))
    t1, t2 = _inverse_moments(U, (sketch.haar_matrix(n, m, seed=11, t=t) for t in range(N)))
    assert abs(t1.mean() - theory.theta1_haar_exact(n, d, m)) <= 4 * t1.std() / np.sqrt(N)
    assert abs(t2.mean() - theory.theta2_haar_exact(n, d, m)) <= 4 * t2.std() / np.sqrt(N)
    # the closed form against a plain evaluation of its own Wishart derivation at another size
    n, d, m = 12, 2, 8
    k = n - m
    e_xi = 1.0 / (m - d - 1)
    D = (m - d) * (m - d - 1) * (m - d - 3)
    e_tr_x2 = d * (m - 1) / D               # E tr X^{-2}
    e_trx_sq = d * ((m - d - 2) * d + 2) / D  # E (tr X^{-1})^2
    tr = d + 2 * k * d * e_xi + k * (k + 1) * e_tr_x2 + k * e_trx_sq
    assert abs(theory.theta2_haar_exact(n, d, m) - tr / d) <= 1e-14 * tr


def test_haar_approximations_are_the_large_size_limit():
    """Section 2's finite-sample approximations against the exact moments.  At (40000, 10000, 20000)
    dropping d^2 moves theta_2 by -20 %, dropping 2 d m by +80 %, a square for the cube by -50 %; the
    approximation itself is within 3e-4 of the exact value, and its error falls like 1/(m - d)."""
    errs = []
    for n, d, m in [(4000, 1000, 2000), (40000, 10000, 20000), (400000, 100000, 200000)]:
        a1, a2 = theory.theta_haar(n, d, m)
        r1 = a1 / theory.theta1_haar_exact(n, d, m) - 1.0
        r2 = a2 / theory.theta2_haar_exact(n, d, m) - 1.0
        assert abs(r1) <= 4.0 / (m - d) and abs(r2) <= 4.0 / (m - d), (n, d, m, r1, r2)
        errs.append(abs(r2))
    assert errs[0] > 5 * errs[1] > 25 * errs[2]


def test_srht_inverse_moments_scaled():
    from oracle import draws
    Nn, d, m, N = 256, 4, 64, 3000
    U, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((Nn, d)))
    t1, t2 = _inverse_moments(U, (sketch.srht_matrix(Nn, m, seed=13, t=t) for t in range(N)))
    c = m / Nn
    e1, e2 = c * theory.theta1_haar_exact(Nn, d, m), c * c * theory.theta2_haar_exact(Nn, d, m)
    # the SRHT follows the Haar trace formulas closely already at this size (observed within 0.1 %);
    # the band is 4 standard errors or 2 %, while a scale of c instead of c^2 would be off by 4x
    assert abs(t1.mean() - e1) <= max(4 * t1.std() / np.sqrt(N), 0.02 * e1)
    assert abs(t2.mean() - e2) <= max(4 * t2.std() / np.sqrt(N), 0.02 * e2)
    assert draws.padded_length(Nn) == Nn
    # the library's rescaled Section 2 values are the same rescaling of the large-size limit
    for NN, dd, mm in [(4096, 1000, 2048), (1 << 16, 10000, 20000)]:
        s1, s2 = theory.srht_thetas_scaled(NN, dd, mm)
        cc = mm / NN
        r1 = s1 / (cc * theory.theta1_haar_exact(NN, dd, mm)) - 1.0
        r2 = s2 / (cc * cc * theory.theta2_haar_exact(NN, dd, mm)) - 1.0
        assert abs(r1) <= 4.0 / (mm - dd) and abs(r2) <= 4.0 / (mm - dd), (NN, dd, mm, r1, r2)
