"""Synthetic tall least-squares problems min ||A x - y||, n >> d.

Recipe (the workloads of the paper are dense tall A with a prescribed spectrum; dimensions are not
printed, so they are set by the caller):
  A = U diag(s) V^T, U (n x d) and V (d x d) orthonormalised from seeded Gaussians,
  s_i = kappa^{-(i-1)/(d-1)}, i = 1..d (geometric from 1 to 1/kappa),
  x_true ~ N(0, I_d),  y = A x_true + sigma * noise.

make_problem   the recipe as stated; the exact minimiser is not known in closed form.
make_planted   the same spectrum, with rows in +-pairs so that the noise can be made exactly
               orthogonal to range(A) *for the stored matrix* (in FP64 or FP32): x* = x_true up to
               the rounding of y, at any n and condition number, with no O(n d^2) solve.
               Rows: A[pi(i)] = b_i and A[pi(h + i)] = D_i b_i (h = n/2, pi a random permutation,
               D_i = +-1), noise z[pi(i)] = w_i, z[pi(h + i)] = -D_i w_i; then A^T z = 0 exactly.
               With b_i = u_i diag(s) V^T / sqrt(2) and U_h orthonormal, A = U' diag(s) V^T with
               U' = P [U_h; D U_h] / sqrt(2) orthonormal.
"""
import concurrent.futures as cf
import os

import numpy as np

CHUNK = 1 << 16


def singular_values(d, kappa):
    i = np.arange(d, dtype=np.float64)
    return kappa ** (-i / max(d - 1, 1))


def _rng(*key):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _orthonormal_columns(Z):
    Q, R = np.linalg.qr(Z)
    return Q * np.where(np.diag(R) < 0, -1.0, 1.0)[None, :]


def make_problem(n, d, kappa, sigma=0.01, seed=0, noise=True):
    """The plain recipe.  Returns dict(A, y, x_true, s, U, V)."""
    if n < d:
        raise ValueError("needs n >= d")
    rng = _rng(seed, 11)
    U = _orthonormal_columns(rng.standard_normal((n, d)))
    V = _orthonormal_columns(rng.standard_normal((d, d)))
    s = singular_values(d, kappa)
    A = (U * s[None, :]) @ V.T
    x_true = rng.standard_normal(d)
    y = A @ x_true
    if noise:
        y = y + sigma * rng.standard_normal(n)
    return dict(A=np.ascontiguousarray(A), y=y, x_true=x_true, s=s, U=U, V=V)


def _threads():
    return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))


def make_planted(n, d, kappa, sigma=0.01, seed=0, want64=True, want32=False):
    """Planted problem with exactly known minimiser x_star = x_true (see the module docstring).
    Returns dict(A64, y64, A32, y32, x_star, s): A64/y64 when want64, A32 (float32) and y32
    (for A32 promoted exactly to FP64) when want32.  Work O(n d^2) in BLAS, O(n d) memory."""
    if n % 2 or n < 2 * d:
        raise ValueError("needs even n >= 2d")
    h = n // 2
    rng = _rng(seed, 21)
    V = _orthonormal_columns(rng.standard_normal((d, d)))
    s = singular_values(d, kappa)
    x_true = rng.standard_normal(d)
    perm = rng.permutation(n)
    D = np.where(rng.random(h) < 0.5, -1.0, 1.0)
    w = _rng(seed, 23).standard_normal(h)
    chunks = [(c0, min(h, c0 + CHUNK)) for c0 in range(0, h, CHUNK)]

    Z = np.empty((h, d))

    def gen(ci):
        c0, c1 = chunks[ci]
        _rng(seed, 22, ci).standard_normal((c1 - c0, d), out=Z[c0:c1])

    with cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(gen, range(len(chunks))))
    # Orthonormalise the Gaussian block: U_h = Z R^{-1} with R^T R = Z^T Z (Z is within a few
    # percent of orthonormal after scaling, so the Gram route loses nothing here).
    G = Z.T @ Z
    R = np.linalg.cholesky(G).T
    Mx = np.linalg.solve(R, s[:, None] * V.T) / np.sqrt(2.0)  # b_i = z_i Mx = u_i diag(s) V^T / sqrt 2

    A64 = np.empty((n, d)) if want64 else None
    A32 = np.empty((n, d), dtype=np.float32) if want32 else None
    top, bot = perm[:h], perm[h:]
    for c0, c1 in chunks:
        B = Z[c0:c1] @ Mx
        if want64:
            A64[top[c0:c1]] = B
            A64[bot[c0:c1]] = D[c0:c1, None] * B
        if want32:
            B32 = B.astype(np.float32)
            A32[top[c0:c1]] = B32
            A32[bot[c0:c1]] = D[c0:c1, None].astype(np.float32) * B32
    del Z
    z = np.empty(n)
    z[top] = w
    z[bot] = -D * w
    out = dict(x_star=x_true, s=s, V=V)
    if want64:
        out["A64"] = A64
        out["y64"] = _matvec(A64, x_true) + sigma * z
    if want32:
        out["A32"] = A32
        out["y32"] = _matvec(A32, x_true) + sigma * z
    return out


def _matvec(A, x):
    """A x in FP64 (FP32 A promoted exactly), by row chunks."""
    y = np.empty(A.shape[0])
    for r0 in range(0, A.shape[0], CHUNK):
        y[r0:r0 + CHUNK] = A[r0:r0 + CHUNK].astype(np.float64, copy=False) @ x
    return y


def make_integer_matrix(n, d, amax, seed=0):
    """n x d int8 matrix with entries uniform on {-amax, ..., amax} (amax <= 127), by row chunks.
    With small integers every partial sum of a signed transform stays an exact integer in FP32 as long
    as amax * n < 2^24, which turns floating-point parity checks into exact ones."""
    if not 0 < amax <= 127:
        raise ValueError("needs 0 < amax <= 127")
    A = np.empty((n, d), dtype=np.int8)
    chunks = [(c0, min(n, c0 + CHUNK)) for c0 in range(0, n, CHUNK)]

    def gen(ci):
        c0, c1 = chunks[ci]
        A[c0:c1] = _rng(seed, 31, ci).integers(-amax, amax + 1, size=(c1 - c0, d), dtype=np.int8)

    with cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(gen, range(len(chunks))))
    return A
