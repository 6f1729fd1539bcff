"""Explicit sketches S A for the three embeddings of Section 2.

Oracle module (test infrastructure only).  Scaling conventions, so that E[S^T S] = I for all three:
  SRHT  S = m^{-1/2} R H_N E with the unnormalised +-1 Sylvester Hadamard matrix
        H_N[k, j] = (-1)^popcount(k & j), A zero-padded to N = 2^ceil(log2 n) rows.
  SJLT  entries +-1/sqrt(s), s per column.
  Gauss entries N(0, 1/m).
"""
import numpy as np

from . import draws


def fwht_rows(X):
    """Walsh-Hadamard transform along axis 0 in Sylvester (natural) order, by log2(N) stages of
    butterflies (u, v) -> (u + v, u - v) on pairs of rows whose indices differ in one bit."""
    X = np.array(X, dtype=np.float64, copy=True)
    N = X.shape[0]
    if N & (N - 1):
        raise ValueError("length must be a power of two")
    h = 1
    while h < N:
        Y = X.reshape(N // (2 * h), 2, h, *X.shape[1:])
        u = Y[:, 0].copy()
        v = Y[:, 1].copy()
        Y[:, 0] = u + v
        Y[:, 1] = u - v
        X = Y.reshape(X.shape)
        h *= 2
    return X


def hadamard_entry(k, j):
    """H_N[k, j] = (-1)^popcount(k & j) for integer arrays k, j."""
    x = np.bitwise_and(np.asarray(k, dtype=np.int64), np.asarray(j, dtype=np.int64))
    return np.where(np.bitwise_count(x) % 2 == 1, -1.0, 1.0)


def srht_sketch(A, m, seed, t=0):
    """S A for the SRHT: sign flip, zero pad, full FWHT, keep the selected rows, scale."""
    n, d = A.shape
    N = draws.padded_length(n)
    e = draws.srht_signs(seed, t, N)
    X = np.zeros((N, d))
    X[:n] = A * e[:n, None]
    Y = fwht_rows(X)
    rows = draws.srht_rows(seed, t, N, m)
    return Y[rows] / np.sqrt(m)


def srht_sketch_rows(A, m, seed, t, which, cols=None, row_block=1 << 16):
    """Selected output rows `which` (positions in [0, m)) of S A, computed directly from the definition
    m^{-1/2} sum_j H_N[k, j] e_j A[j, cols] (for spot checks at large n): the +-1 coefficients of those
    rows are formed explicitly for a block of rows j of A at a time and multiplied with that block
    (A may be of any real or integer dtype; the block is promoted to FP64)."""
    n, d = A.shape
    N = draws.padded_length(n)
    cols = np.arange(d) if cols is None else np.asarray(cols)
    e = draws.srht_signs(seed, t, N)[:n]
    k = draws.srht_rows(seed, t, N, m)[np.asarray(which)]
    out = np.zeros((len(k), len(cols)))
    for j0 in range(0, n, row_block):
        j1 = min(n, j0 + row_block)
        coef = hadamard_entry(k[:, None], np.arange(j0, j1)[None, :]) * e[None, j0:j1]
        out += coef @ np.asarray(A[j0:j1][:, cols], dtype=np.float64)
    return out / np.sqrt(m)


def srht_matrix(n, m, seed, t=0):
    """Dense S (m x N) of the SRHT (small N only)."""
    N = draws.padded_length(n)
    e = draws.srht_signs(seed, t, N)
    rows = draws.srht_rows(seed, t, N, m)
    j = np.arange(N)
    H = hadamard_entry(rows[:, None], j[None, :])
    return H * e[None, :] / np.sqrt(m)


def sjlt_matrix(n, m, s, seed, t=0):
    """Dense S (m x n) of the SJLT."""
    tg, sg = draws.sjlt_draws(seed, t, n, m, s)
    S = np.zeros((m, n))
    for k in range(s):
        S[tg[:, k], np.arange(n)] = sg[:, k] / np.sqrt(s)
    return S


def sjlt_sketch(A, m, s, seed, t=0):
    """S A for the SJLT as a scatter-add of signed rows of A into their target rows."""
    n, d = A.shape
    tg, sg = draws.sjlt_draws(seed, t, n, m, s)
    SA = np.zeros((m, d))
    for k in range(s):
        np.add.at(SA, tg[:, k], A * (sg[:, k] / np.sqrt(s))[:, None])
    return SA


def gaussian_sketch(A, m, seed, t=0, row_block=4096):
    """S A for the Gaussian embedding, generating S in blocks of columns (rows of A)."""
    n, d = A.shape
    SA = np.zeros((m, d))
    for j0 in range(0, n, row_block):
        j1 = min(n, j0 + row_block)
        S = draws.gaussian_normals(seed, t, np.arange(m)[:, None], np.arange(j0, j1)[None, :]) / np.sqrt(m)
        SA += S @ A[j0:j1]
    return SA


def gaussian_sketch_bf16(A, m, seed, t=0, row_block=4096):
    """S A for the precision form of the Gaussian embedding: the standard normals are rounded to
    bfloat16 before scaling by 1/sqrt(m) (the product with A in float64)."""
    n, d = A.shape
    SA = np.zeros((m, d))
    for j0 in range(0, n, row_block):
        j1 = min(n, j0 + row_block)
        G = draws.round_bf16(draws.gaussian_normals(seed, t, np.arange(m)[:, None], np.arange(j0, j1)[None, :]))
        SA += G @ A[j0:j1]
    return SA / np.sqrt(m)


def haar_matrix(n, m, seed, t=0):
    """S (m x n) of the Haar embedding (Section 2): orthonormal rows, S S^T = I_m, spanning a uniformly
    distributed m-dimensional subspace.  S = Q^T for the QR factorization G = Q R with a positive
    diagonal of R, where G (n x m) holds the Gaussian embedding's standard normals, G[j, i] = g(i, j);
    Q is then Haar distributed (the positive-diagonal convention makes the factorization unique).
    Rows are not rescaled: the inverse moments of C_S for this S are the Haar ones of Section 2."""
    G = draws.gaussian_normals(seed, t, np.arange(m)[None, :], np.arange(n)[:, None])
    Q, R = np.linalg.qr(G)
    return (Q * np.sign(np.diag(R))[None, :]).T


def haar_sketch(A, m, seed, t=0):
    """S A for the Haar embedding (dense S; small n only)."""
    return haar_matrix(A.shape[0], m, seed, t) @ A


def sketch(A, kind, m, seed, t=0, s=1):
    if kind == "haar":
        return haar_sketch(A, m, seed, t)
    if kind == "srht":
        return srht_sketch(A, m, seed, t)
    if kind == "sjlt":
        return sjlt_sketch(A, m, s, seed, t)
    if kind == "gaussian":
        return gaussian_sketch(A, m, seed, t)
    raise ValueError(kind)
