"""Householder QR and triangular solves, written out as in the textbook algorithm
(Golub & Van Loan, Matrix Computations, Algorithm 5.2.1): for k = 0..d-1 reflect column k onto
a multiple of e_k and apply the reflector to the trailing columns.

Oracle module (test infrastructure only).  Used for the direct least-squares solve and for the
preconditioner factor of Section 1.2 (H_S = R^T R with R from the QR of S A; the paper allows
QR of S A or a Cholesky factor of H_S).  R is sign-normalised so that diag(R) > 0, which makes it
unique for a full-rank input.
"""
import numpy as np


def householder_qr(X, extra=None):
    """Upper-triangular R (d x d, positive diagonal) of X (rows >= cols).  If `extra` (a vector or
    a matrix with as many rows as X) is given, Q^T extra is returned as well."""
    R = np.array(X, dtype=np.float64, copy=True)
    rows, d = R.shape
    if rows < d:
        raise ValueError("QR needs rows >= cols")
    E = None if extra is None else np.array(extra, dtype=np.float64, copy=True)
    for k in range(d):
        x = R[k:, k]
        nx = np.sqrt(np.dot(x, x))
        if nx == 0.0:
            continue
        alpha = -nx if x[0] >= 0 else nx  # reflect away from x to avoid cancellation
        v = x.copy()
        v[0] -= alpha
        vv = np.dot(v, v)
        if vv == 0.0:
            continue
        tau = 2.0 / vv
        R[k:, k:] -= tau * np.outer(v, v @ R[k:, k:])
        if E is not None:
            E[k:] -= tau * (np.outer(v, v @ E[k:]) if E.ndim == 2 else v * np.dot(v, E[k:]))
    R = np.triu(R[:d])
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    R = sgn[:, None] * R
    if E is None:
        return R
    E = E[:d] * (sgn[:, None] if E.ndim == 2 else sgn)
    return R, E


def tsqr(row_blocks):
    """R and Q^T y of a tall system given as an iterable of (A_block, y_block): QR every block,
    stack the small triangular factors, QR again (the same mathematics as one Householder QR,
    with memory proportional to one block)."""
    Rs, cs = [], []
    for Ab, yb in row_blocks:
        if Ab.shape[0] < Ab.shape[1]:
            Rs.append(Ab)
            cs.append(yb)
            continue
        R, c = householder_qr(Ab, yb)
        Rs.append(R)
        cs.append(c)
    return householder_qr(np.vstack(Rs), np.concatenate(cs))


def back_substitute(R, c):
    """Solve R x = c for upper-triangular R, last row first."""
    d = R.shape[0]
    x = np.zeros(d)
    for i in range(d - 1, -1, -1):
        x[i] = (c[i] - np.dot(R[i, i + 1:], x[i + 1:])) / R[i, i]
    return x


def forward_substitute_transposed(R, c):
    """Solve R^T z = c for upper-triangular R, first row first."""
    d = R.shape[0]
    z = np.zeros(d)
    for i in range(d):
        z[i] = (c[i] - np.dot(R[:i, i], z[:i])) / R[i, i]
    return z
