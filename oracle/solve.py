"""Direct least-squares solve x* = argmin ||A x - y||_2 and the error metrics.

Oracle module (test infrastructure only).  The problem is f(x) = 1/2 <x, H x> - <b, x> with
H = A^T A (Section 1); for least squares b = A^T y, so the minimiser is the least-squares solution.
The direct solve is Householder QR of [A | y] followed by back-substitution (no normal equations).

Error metrics (Section 1.5 notation): delta_t = 1/2 ||x_t - x*||_H^2 = 1/2 ||A (x_t - x*)||^2;
the relative A-norm error is e_A(x) = ||A (x - x*)|| / ||A x*||, so delta_t / delta_0 = e_A^2
for the start point x_0 = 0.
"""
import numpy as np

from .householder import back_substitute, householder_qr, tsqr


def lstsq_householder(A, y, block_rows=None):
    """x* by Householder QR (TSQR over row blocks of `block_rows` rows when given)."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if block_rows is None or block_rows >= A.shape[0]:
        R, c = householder_qr(A, y)
    else:
        blocks = ((A[i:i + block_rows], y[i:i + block_rows]) for i in range(0, A.shape[0], block_rows))
        R, c = tsqr(blocks)
    return back_substitute(R, c)


def a_norm_error(A, x, x_ref):
    """e_A(x) = ||A (x - x_ref)|| / ||A x_ref||."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A @ (x - x_ref)) / np.linalg.norm(A @ x_ref))


def normal_equation_residual(A, x, y):
    """||A^T (A x - y)|| / (||A||_2 ||A x - y||): zero at the exact minimiser."""
    r = A @ x - y
    return float(np.linalg.norm(A.T @ r) / (np.linalg.norm(A, 2) * np.linalg.norm(r)))


def min_norm_lstsq(A, y, rcond=1e-12):
    """x+ = V Sigma^+ U^T y, the minimum-norm least-squares solution (singular values at or below
    rcond * sigma_max treated as zero), from numpy's SVD of A."""
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    keep = s > rcond * s[0]
    return Vt[keep].T @ ((U[:, keep].T @ np.asarray(y, dtype=np.float64)) / s[keep])

