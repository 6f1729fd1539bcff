"""Preconditioned conjugate gradient with a fixed sketch (Section 1.2), written step by step.

Oracle module (test infrastructure only).

With H = A^T A, b = A^T y and the sketched Hessian H_S = (S A)^T (S A) = R^T R:
    r_0 = b - H x_0,  solve H_S rhat_0 = r_0,  p_0 = rhat_0
    alpha_t = r_t^T rhat_t / p_t^T H p_t
    x_{t+1} = x_t + alpha_t p_t,   r_{t+1} = r_t - alpha_t H p_t
    solve H_S rhat_{t+1} = r_{t+1}
    p_{t+1} = rhat_{t+1} + (r_{t+1}^T rhat_{t+1} / r_t^T rhat_t) p_t
H p is formed as A^T (A p); H_S^{-1} r as R^{-1} (R^{-T} r) by two triangular substitutions.

Stop rule: rho_t = r_t^T rhat_t equals Delta_t^T C_S^{-1} Delta_t (Section 1.5 notation), so when the
eigenvalues of C_S lie in an interval of ratio at most 16 the relative A-norm error is at most
4 sqrt(rho_t / rho_0) (for x_0 = 0).  The solve stops once sqrt(rho_t / rho_0) <= tol / 4.
"""
import numpy as np

from . import sketch as _sk
from .householder import back_substitute, forward_substitute_transposed, householder_qr


def apply_hs_inv(R, r):
    return back_substitute(R, forward_substitute_transposed(R, r))


def sketch_factor(A, kind, m, seed, t=0, s=1):
    """R (upper triangular, positive diagonal) with H_S = R^T R, from the QR of S A."""
    return householder_qr(_sk.sketch(A, kind, m, seed, t, s))


def svd_preconditioner(SA, rtol=1e-12):
    """P = V Sigma^+ from numpy's SVD of S A (singular values at or below rtol * sigma_max dropped), so
    that P P^T = H_S^+ (the LSRN form of the factor step; equal to R^{-1} R^{-T} for full-rank S A)."""
    _, s, Vt = np.linalg.svd(np.asarray(SA, dtype=np.float64), full_matrices=False)
    keep = s > rtol * s[0]
    return Vt[keep].T / s[keep][None, :]


def qrcp_preconditioner(SA, rtol=1e-12):
    """W = P [R11^{-1}; 0] from scipy's column-pivoted QR S A P = Q R, R11 the leading r x r block with
    |R_kk| > rtol |R_00|: W W^T = H_S^{-1} at full rank, and the basic solution on the kept columns
    otherwise.  Returns (W, r, piv)."""
    import scipy.linalg
    SA = np.asarray(SA, dtype=np.float64)
    d = SA.shape[1]
    _, R, piv = scipy.linalg.qr(SA, mode="economic", pivoting=True)
    diag = np.abs(np.diag(R))
    r = int(np.sum(diag > rtol * diag[0])) if diag[0] > 0 else 0
    W = np.zeros((d, d))
    W[piv[:r], :r] = np.linalg.inv(np.triu(R[:r, :r]))
    return W, r, piv


def pcg(A, y, R, x0=None, tol=1e-10, max_iter=200, fixed_iters=None):
    """Run PCG.  Returns (x, iterates) where iterates[t] = x_t.  With fixed_iters the loop runs
    exactly that many iterations; otherwise it stops by the rule in the module docstring."""
    return pcg_with(A, y, lambda r: apply_hs_inv(R, r), x0, tol, max_iter, fixed_iters)


def pcg_svd(A, y, P, x0=None, tol=1e-10, max_iter=200, fixed_iters=None):
    """PCG with the preconditioner P P^T (svd_preconditioner)."""
    return pcg_with(A, y, lambda r: P @ (P.T @ r), x0, tol, max_iter, fixed_iters)


def pcg_with(A, y, hs_inv, x0=None, tol=1e-10, max_iter=200, fixed_iters=None):
    """The PCG loop with H_S^{-1} (or H_S^+) applied by hs_inv."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    x = np.zeros(d) if x0 is None else np.array(x0, dtype=np.float64)
    r = A.T @ (y - A @ x)
    rhat = hs_inv(r)
    p = rhat.copy()
    rho = float(r @ rhat)
    rho0 = rho
    iterates = [x.copy()]
    iters = max_iter if fixed_iters is None else fixed_iters
    for _ in range(iters):
        if fixed_iters is None and (rho0 == 0.0 or np.sqrt(max(rho, 0.0) / rho0) <= tol / 4):
            break
        q = A @ p
        Hp = A.T @ q
        pHp = float(q @ q)
        if pHp <= 0.0:
            break
        alpha = rho / pHp
        x = x + alpha * p
        r = r - alpha * Hp
        rhat = hs_inv(r)
        rho_new = float(r @ rhat)
        p = rhat + (rho_new / rho) * p
        rho = rho_new
        iterates.append(x.copy())
    return x, iterates


def pcg_solve(A, y, kind, m, seed, s=1, tol=1e-10, max_iter=200):
    R = sketch_factor(A, kind, m, seed, 0, s)
    return pcg(A, y, R, tol=tol, max_iter=max_iter)
