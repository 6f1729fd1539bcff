"""Pins of the oracle's flexible conjugate gradient (FCG / GCC / IPCG) with refreshed sketches:
  Section 1.2        with a fixed sketch every window k >= 1 reproduces PCG (the directions of CG with
                     a fixed preconditioner are conjugate to all earlier ones)
  conjugate directions
                     GCC (full window) with fresh sketches ends at x* after d steps
  Section 4          FCG improves locally on the IHS step: from the same x_t and S_t, the new error
                     is at most the best error along v_t = H_{S_t}^{-1} r_t
  Corollary 4.2      E delta_t / E delta_0 <= (1 - theta_1^2 / theta_2)^t for refreshed Gaussian
                     embeddings (Monte Carlo over sketch seeds)
"""
import numpy as np
import pytest

from oracle import theory
from oracle.fcg import fcg
from oracle.householder import householder_qr
from oracle.pcg import apply_hs_inv, pcg, sketch_factor
from oracle import sketch as sk
from oracle.solve import lstsq_householder
from synth import make_problem


def _delta(A, x, xs):
    return 0.5 * float(np.sum((A @ (x - xs)) ** 2))


@pytest.mark.parametrize("kind", ["gaussian", "srht", "sjlt"])
def test_fixed_sketch_fcg_is_pcg(kind):
    n, d, m, T = 512, 12, 48, 8
    P = make_problem(n, d, 1e3, seed=21)
    A, y = P["A"], P["y"]
    R = sketch_factor(A, kind, m, 9, 0, 2)
    _, ref = pcg(A, y, R, fixed_iters=T)
    scale = float(np.linalg.norm(A @ lstsq_householder(A, y)))
    for k in (1, 2, T):
        its = fcg(A, y, kind, m, seed=9, k=k, iters=T, refresh=False, s=2)
        for t in range(T + 1):
            assert np.linalg.norm(A @ (its[t] - ref[t])) <= 1e-9 * scale, (k, t)
    # without conjugation (k = 0) the method is a line-searched IHS, which is slower than PCG
    ihs_ls = fcg(A, y, kind, m, seed=9, k=0, iters=T, refresh=False, s=2)
    xs = lstsq_householder(A, y)
    assert _delta(A, ihs_ls[T], xs) > 2.0 * _delta(A, ref[T], xs)


def test_gcc_terminates_in_d_steps_with_fresh_sketches():
    n, d, m = 256, 6, 24
    P = make_problem(n, d, 1e3, seed=22)
    A, y = P["A"], P["y"]
    xs = lstsq_householder(A, y)
    d0 = _delta(A, np.zeros(d), xs)
    for kind in ("gaussian", "srht", "sjlt"):
        gcc = fcg(A, y, kind, m, seed=31, k=d, iters=d, s=2)
        assert _delta(A, gcc[d], xs) <= 1e-20 * d0, kind
        # the truncated windows do not terminate (fresh sketches break the conjugacy they skip)
        ipcg = fcg(A, y, kind, m, seed=31, k=1, iters=d, s=2)
        assert _delta(A, ipcg[d], xs) > 1e-12 * d0, kind


@pytest.mark.parametrize("k", [1, 2, 50])
def test_fcg_step_beats_best_ihs_step_from_same_point(k):
    n, d, m, T = 1024, 16, 40, 12
    P = make_problem(n, d, 1e4, seed=23)
    A, y = P["A"], P["y"]
    xs = lstsq_householder(A, y)
    its = fcg(A, y, "gaussian", m, seed=41, k=k, iters=T)
    for t in range(T):
        x = its[t]
        R = householder_qr(sk.sketch(A, "gaussian", m, 41, t))
        r = A.T @ (y - A @ x)
        v = apply_hs_inv(R, r)
        Av = A @ v
        mu = float(v @ r) / float(Av @ Av)  # exact line search along v_t
        best_ihs = _delta(A, x + mu * v, xs)
        assert _delta(A, its[t + 1], xs) <= best_ihs * (1 + 1e-9) + 1e-300, t


def test_refreshed_gaussian_fcg_within_corollary_4_2_bound():
    n, d, m, T, reps = 1024, 16, 48, 10, 32
    P = make_problem(n, d, 1e5, seed=24)
    A, y = P["A"], P["y"]
    xs = lstsq_householder(A, y)
    t1, t2 = theory.theta_gaussian(m, d)
    bound = (1.0 - t1 * t1 / t2) ** np.arange(T + 1)
    for k in (1, T):
        sims = np.array([[_delta(A, x, xs) for x in fcg(A, y, "gaussian", m, seed=700 + r, k=k, iters=T)]
                         for r in range(reps)])
        sims /= sims[:, :1]
        mean = sims.mean(axis=0)
        se = sims.std(axis=0) / np.sqrt(reps)
        # the expectation is below the bound; allow 4 standard errors of Monte Carlo noise
        assert np.all(mean[1:] <= bound[1:] + 4 * se[1:]), k
        # and the flexible method is strictly faster than the bound by the end
        assert mean[T] < bound[T]
