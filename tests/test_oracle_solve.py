"""Pins of the oracle's direct solve and QR: planted noise-free solutions, the normal-equation
invariant, exact rational arithmetic on tiny inputs, LAPACK's SVD-based solver within the FP64
conditioning floor, and the defining properties of the R factor."""
from fractions import Fraction

import numpy as np

from oracle.householder import householder_qr, back_substitute, forward_substitute_transposed
from oracle.solve import a_norm_error, lstsq_householder, normal_equation_residual
from synth import make_planted, make_problem

U64 = np.finfo(np.float64).eps / 2


def test_planted_noise_free():
    for kappa in (1e2, 1e6, 1e8):
        P = make_problem(600, 12, kappa, seed=1, noise=False)
        x = lstsq_householder(P["A"], P["y"])
        assert a_norm_error(P["A"], x, P["x_true"]) < 1e-13


def test_planted_orthogonal_noise_and_tsqr():
    P = make_planted(4000, 16, 1e3, sigma=0.01, seed=2)
    x1 = lstsq_householder(P["A64"], P["y64"])
    x2 = lstsq_householder(P["A64"], P["y64"], block_rows=512)
    assert a_norm_error(P["A64"], x1, P["x_star"]) < 1e-12
    assert a_norm_error(P["A64"], x2, P["x_star"]) < 1e-12


def test_normal_equation_invariant():
    for kappa in (1e4, 1e6):
        P = make_problem(2000, 20, kappa, seed=3)
        x = lstsq_householder(P["A"], P["y"])
        assert normal_equation_residual(P["A"], x, P["y"]) < 20 * U64 * kappa


def test_brute_force_rational():
    rng = np.random.default_rng(4)
    for trial in range(6):
        n, d = int(rng.integers(4, 9)), int(rng.integers(1, 4))
        A = rng.integers(-5, 6, size=(n, d)).astype(float)
        if np.linalg.matrix_rank(A) < d:
            continue
        y = rng.integers(-9, 10, size=n).astype(float)
        # exact normal equations (A^T A) x = A^T y by Gauss-Jordan over the rationals
        M = [[Fraction(int(sum(A[k, i] * A[k, j] for k in range(n)))) for j in range(d)]
             + [Fraction(int(sum(A[k, i] * y[k] for k in range(n))))] for i in range(d)]
        for c in range(d):
            piv = next(r for r in range(c, d) if M[r][c] != 0)
            M[c], M[piv] = M[piv], M[c]
            M[c] = [v / M[c][c] for v in M[c]]
            for r in range(d):
                if r != c and M[r][c] != 0:
                    f = M[r][c]
                    M[r] = [a - f * b for a, b in zip(M[r], M[c])]
        exact = np.array([float(M[i][d]) for i in range(d)])
        x = lstsq_householder(A, y)
        assert np.max(np.abs(x - exact)) <= 1e-13 * max(1.0, np.max(np.abs(exact)))


def test_against_lapack_within_floor():
    P = make_problem(3000, 24, 1e5, seed=5)
    x = lstsq_householder(P["A"], P["y"])
    xl = np.linalg.lstsq(P["A"], P["y"], rcond=None)[0]
    r = P["A"] @ xl - P["y"]
    floor = U64 * 1e5 * np.linalg.norm(r) / np.linalg.norm(P["A"] @ xl)
    assert a_norm_error(P["A"], x, xl) < 50 * floor


def test_qr_factor_properties():
    X = np.random.default_rng(6).standard_normal((40, 7))
    R = householder_qr(X)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(R.T @ R, X.T @ X, rtol=1e-13, atol=1e-12)
    # unique positive-diagonal R: equals the Cholesky factor of the Gram
    assert np.allclose(R, np.linalg.cholesky(X.T @ X).T, atol=1e-12)
    c = np.arange(7.0)
    assert np.allclose(R @ back_substitute(R, c), c)
    assert np.allclose(R.T @ forward_substitute_transposed(R, c), c)
