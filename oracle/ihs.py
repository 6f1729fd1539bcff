"""Iterative Hessian sketch and its heavy-ball variant (Section 1.1), step by step.

Oracle module (test infrastructure only).

    IHS          x_{t+1} = x_t - mu H_{S_t}^{-1} grad f(x_t)
    Polyak-IHS   x_{t+1} = x_t - mu H_{S_t}^{-1} grad f(x_t) + beta (x_t - x_{t-1})
with grad f(x) = H x - b = A^T (A x - y), H_{S_t} = R_t^T R_t from the QR of S_t A, and x_{-1} = x_0
(so the first step is a plain IHS step).  Refreshed: S_t is drawn with refresh counter t (fresh,
independent draws every iteration, Section 4).  Fixed: S_t = S_0 for all t (Section 3).
"""
import numpy as np

from .householder import householder_qr
from .pcg import apply_hs_inv
from . import sketch as _sk


def ihs(A, y, kind, m, seed, mu, beta=0.0, iters=20, refresh=True, s=1, x0=None):
    """Returns the iterates [x_0, ..., x_iters]."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    x = np.zeros(d) if x0 is None else np.array(x0, dtype=np.float64)
    x_prev = x.copy()
    R_fixed = None if refresh else householder_qr(_sk.sketch(A, kind, m, seed, 0, s))
    out = [x.copy()]
    for t in range(iters):
        R = householder_qr(_sk.sketch(A, kind, m, seed, t, s)) if refresh else R_fixed
        g = A.T @ (A @ x - y)
        x_next = x - mu * apply_hs_inv(R, g) + beta * (x - x_prev)
        x_prev, x = x, x_next
        out.append(x.copy())
    return out
