"""Flexible conjugate gradient with refreshed sketches (Section 1.2, Section 4), step by step.

Oracle module (test infrastructure only).

With H = A^T A, the negative gradient r_t = A^T (y - A x_t) and a sketch S_t drawn with refresh
counter t (H_{S_t} = R_t^T R_t from the QR of S_t A):
    v_t = H_{S_t}^{-1} r_t
    p_t = v_t - sum_{j = t - k_t}^{t - 1} (<v_t, H p_j> / <p_j, H p_j>) p_j
    alpha_t = <p_t, r_t> / <p_t, H p_t>
    x_{t+1} = x_t + alpha_t p_t
with the conjugation window k_t = min(k, t), so that 0 <= k_{t+1} <= k_t + 1 as the method requires:
k >= the number of iterations is GCC (every earlier direction), k = 1 is IPCG, k = 0 is the IHS
step along v_t with an exact line search.

Readings: the direction is built from -grad f, which flips the sign of every p_t relative to the
paper's v_t = H_S^{-1} grad f and leaves alpha_t p_t unchanged; the step length is the exact line
search <p_t, r_t> / <p_t, H p_t>, which equals the printed <p_t, b> / <p_t, H p_t> for GCC started
at x_0 = 0 (then <p_t, H x_t> = 0) and is the minimiser along p_t for every window.  A direction
with <p_t, H p_t> = 0 (v_t already in the span of the window) leaves x unchanged and is skipped in
later projections.  <p_j, H p_j> is formed as ||A p_j||^2.
"""
import numpy as np

from .householder import householder_qr
from .pcg import apply_hs_inv
from . import sketch as _sk


def fcg(A, y, kind, m, seed, k, iters=20, refresh=True, s=1, x0=None, t0=0):
    """Returns the iterates [x_0, ..., x_iters].  Sketch t uses refresh counter t0 + t (t0 when
    refresh is False)."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    x = np.zeros(d) if x0 is None else np.array(x0, dtype=np.float64)
    P, HP, PHP = [], [], []  # directions p_j, H p_j and <p_j, H p_j>, oldest first
    R_fixed = None if refresh else householder_qr(_sk.sketch(A, kind, m, seed, t0, s))
    out = [x.copy()]
    for t in range(iters):
        R = householder_qr(_sk.sketch(A, kind, m, seed, t0 + t, s)) if refresh else R_fixed
        r = A.T @ (y - A @ x)
        v = apply_hs_inv(R, r)
        kt = min(k, t)
        p = v.copy()
        for j in range(t - kt, t):
            if PHP[j] > 0.0:
                p -= (float(v @ HP[j]) / PHP[j]) * P[j]
        q = A @ p
        Hp = A.T @ q
        pHp = float(q @ q)
        if pHp > 0.0:
            x = x + (float(p @ r) / pHp) * p
        P.append(p)
        HP.append(Hp)
        PHP.append(pHp)
        out.append(x.copy())
    return out
